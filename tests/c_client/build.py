"""Builds the plain C client of libnpm (npm_client.c, beside this file) with
gcc against include/npm.h, the in-tree libnpm.so and the HIP runtime's C API
only: no Python, no torch.  Run as a script it writes npm_client here."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
PKG = os.path.join(ROOT, "paper_2504_04315_amd")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
BINARY = os.path.join(HERE, "npm_client")


def up_to_date():
    """Whether the in-tree binary exists and is newer than the header and
    the client's source (a stale binary would pass the wrong structures)."""
    if not os.path.exists(BINARY):
        return False
    t = os.path.getmtime(BINARY)
    return all(os.path.getmtime(f) <= t for f in (os.path.join(ROOT, "include", "npm.h"),
                                                   os.path.join(HERE, "npm_client.c")))


def build(out=BINARY):
    cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROCM, "include"),
           os.path.join(HERE, "npm_client.c"), "-o", out,
           "-L", PKG, "-lnpm", "-Wl,-rpath,$ORIGIN/../../paper_2504_04315_amd", f"-Wl,-rpath,{PKG}",
           "-L", os.path.join(ROCM, "lib"), "-lamdhip64", f"-Wl,-rpath,{os.path.join(ROCM, 'lib')}",
           "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"building the C client failed:\n{' '.join(cmd)}\n{r.stderr}")
    return out


if __name__ == "__main__":
    print(build(*sys.argv[1:]))
