"""MI355X-native truncated SVD: augmented, restarted Lanczos bidiagonalization
with full (CGS2) re-orthogonalization, hand-written HIP kernels for gfx950
behind a C ABI (``include/svds.h``).

Submodules are imported on demand: ``inputs`` (seeded synthetic matrices) needs
no GPU; ``svds`` loads the native library and fails loudly if it is missing.
"""
