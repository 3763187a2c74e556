"""CPU checks of arithmetic building blocks the kernels rely on (no GPU needed)."""
import numpy as np


def _fma_sign(a, b, c):
    """Sign of c - a*b for FP32 a, b, c, exactly (the product of two FP32 values and the
    difference with a nearby FP32 value are exact in FP64), as the kernel's fmaf gives it."""
    return np.sign(c.astype(np.float64) - a.astype(np.float64) * b.astype(np.float64))


def _refine(x, s):
    """The kernel's sqrt_rn correction applied to a candidate s within 1 ulp of sqrt(x)."""
    s_dn = (s.view(np.int32) - 1).view(np.float32)
    s_up = (s.view(np.int32) + 1).view(np.float32)
    down = _fma_sign(s_dn, s, x) <= 0
    up = (~down) & (_fma_sign(s_up, s, x) > 0)
    return np.where(down, s_dn, np.where(up, s_up, s))


def test_sqrt_refinement_gives_the_correctly_rounded_root():
    rng = np.random.default_rng(0)
    x = np.concatenate([
        rng.uniform(1e-6, 400.0, 200000).astype(np.float32),
        (np.arange(1, 20001, dtype=np.float32) ** 2),                        # exact squares
        (rng.integers(1, 1 << 12, 20000).astype(np.float32) ** 2 + 1.0).astype(np.float32),
        np.float32(2.0) ** np.arange(-19, 9, dtype=np.float32),
    ]).astype(np.float32)
    exact = np.sqrt(x)              # numpy float32 sqrt is correctly rounded (IEEE)
    for off in (-1, 0, 1):          # the hardware result may be off by one ulp either way
        cand = (exact.view(np.int32) + off).view(np.float32)
        assert np.array_equal(_refine(x, cand), exact), off
