"""MI355X-native SIMPLE-TS time step (arXiv 1802.04243): HIP kernels behind a C ABI."""
