"""FP64 CPU oracle of the projection-based RCA ULM reconstruction path.

TEST INFRASTRUCTURE.  This package exists to prove the GPU path correct.
Only `tests/`, the smoke check in `__graft_entry__.py` and the CPU-baseline
leg of `bench.py` may import it.  It shares no code with the HIP path: the
two meet only through the seeded inputs of the `synth` package.

Every function cites the passage of the paper it follows.  Where the paper is
silent, the reading taken is stated in the function's module docstring.

Modules:
  sim        forward model of the channel data (input generator twin)
  beamform   two-stage beamforming to projection planes; full-3D DAS
  clutter    eigen-based SVD clutter filter; direct SVD route
  localize   envelope, NCC with a Gaussian template, regional peaks, sub-pixel
  pipeline   the whole path; density map; SSIM
  cnn        learned localiser: conv layers, head, loss, Adam (FP64)
  philox     counter-based generator for the channel noise
"""
