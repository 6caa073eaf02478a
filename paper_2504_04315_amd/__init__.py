"""MI355X-native hot path of Neural Parametric Mixtures (NPM) for path guiding.

The compute path is the HIP library ``libnpm.so`` built from ``csrc/`` behind
the C ABI in ``include/npm.h``; :mod:`.npm` is its thin ctypes binding.  The
package import is light: nothing is loaded until a binding object is made.
"""
__all__ = ["npm", "workload"]
