"""MI355X-native DEC beam propagation: z-marching of the nonlinear Schroedinger
equation on unstructured triangular meshes (HIP kernels behind a C ABI)."""
