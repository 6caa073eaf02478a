"""FP64 CPU oracle of the NPM hot path -- test infrastructure only.

Only tests/, the smoke check and the benchmark's CPU-baseline leg import this
package.  The product path (the HIP library and its binding) never does.
"""
