"""MI355X-native MUSCL-Hancock Godunov hydrodynamics hot path (HIP kernels behind a C ABI)."""
