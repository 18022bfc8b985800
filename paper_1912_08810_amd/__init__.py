"""MI355X (gfx950) scattering self-energy library: hand-written HIP kernels
behind a C ABI (include/sse.h), with a thin ctypes binding (``sse``)."""
