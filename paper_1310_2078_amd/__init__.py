"""SL1M hot path on MI355X: the direct measurement operator, its adjoint and
the FISTA solve, as hand-written HIP kernels behind a C ABI (libsl1m.so)."""
