"""MI355X-native Polarized SARA: HIP kernels behind a C ABI, with a thin ctypes binding."""
