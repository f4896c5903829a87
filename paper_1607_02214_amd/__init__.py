"""MI355X-native PPMLR-MHD split-sweep library (HIP kernels behind a C ABI)."""
