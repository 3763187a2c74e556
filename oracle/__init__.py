"""Plain, slow, obviously-correct CPU oracle of the neural visibility cache.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
bench's CPU-baseline leg may import anything from this package; the product
path (the HIP library and its Python binding) never does.  It shares no code
with the HIP path: both consume the same seeded input arrays from
``workloads`` and nothing else.

Arithmetic is FP64 (NumPy) except where floating point decides an integer
result: the grid cell of a position, the light chosen by weighted reservoir
sampling and the binary shadow-ray label.  Those decisions are taken in FP32,
the precision of the kernels, with the operation order stated in each
function, so that both sides reach the same integer.

Modules (paper passages in brackets):
  philox     counter-based generator (Salmon et al. 2011)       [random draws]
  hashgrid   multi-resolution hash-grid encoding                [Sec. 3.1 Fig. overview, Sec. 3.3]
  mlp        visibility MLP forward and backward                [Sec. 3.3, Sec. 3.4]
  lighting   unshadowed weight, clamp, WRS, neural DI           [Sec. 1, Sec. 3.1, Sec. 3.2]
  shadow     shadow-ray labels against sphere occluders         [Sec. 3.4]
  training   loss, pixel selection, table gradient, Adam        [Sec. 3.3, Sec. 3.4]
  estimator  exact moments of the light-sampling estimator      [Sec. 1, Sec. 3.1]
  clustered  k-means clusters, cluster labels, two-step sampling [Sec. 3.6]
  pipeline   the frame composed from the steps above
"""
