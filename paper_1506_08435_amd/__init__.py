"""MI355X (gfx950) non-negative diffusion QP library (arXiv:1506.08435).

`nnqp` is the Python binding of the C ABI in include/nnqp.h (libnnqp.so);
`workloads` builds the seeded synthetic inputs.  Importing the package does
not load the HIP library; creating an `nnqp.Context` does, and fails loudly
if the library is not built.
"""
__all__ = ["nnqp", "workloads"]
