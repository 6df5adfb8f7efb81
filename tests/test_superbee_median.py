"""The FP32 superbee slope of the motor kernel is built from medians (Sec. 2's superbee limiter):
minmod(x, y) = med3(x, y, 0), and the maxmod of p = minmod(2a, b) and q = minmod(a, 2b) is
med3(p, q, 2b), since both lie between 0 and 2b.  Checked here in FP32 against the limiter's
definition, sgn(b) max(min(2|a|, |b|), min(|a|, 2|b|)) where a and b have the same strict sign,
else 0, and against the earlier third operand sgn(b) inf.  CPU only."""
import numpy as np


def med3(x, y, z):
    return np.maximum(np.minimum(x, y), np.minimum(np.maximum(x, y), z))


def superbee_def(a, b):
    aa, ab = np.abs(a), np.abs(b)
    m = np.maximum(np.minimum(aa + aa, ab), np.minimum(aa, ab + ab))
    same = (np.sign(a) == np.sign(b)) & (a != 0)
    return np.where(same, np.copysign(m, b), np.float32(0)).astype(np.float32)


def test_median_form_equals_the_definition():
    rng = np.random.default_rng(7)
    vals = np.concatenate([rng.standard_normal(200000), rng.standard_normal(2000) * 1e-30,
                           rng.standard_normal(2000) * 1e30, [0.0, -0.0, 1.0, -1.0, 2.0, -2.0, 0.5, -0.5]])
    a = rng.permutation(vals).astype(np.float32)
    b = rng.permutation(vals).astype(np.float32)
    edge = np.array([0, 1, 2, 0.5, -1, -2, -0.5, 3], dtype=np.float32)   # ties: 2a = b, a = 2b, a = b
    a = np.concatenate([a, edge, 2 * edge, 0.5 * edge]).astype(np.float32)
    b = np.concatenate([b, edge, edge, edge]).astype(np.float32)
    with np.errstate(over="ignore"):
        b2 = (b + b).astype(np.float32)
        p = med3((a + a).astype(np.float32), b, np.float32(0))
        q = med3(a, b2, np.float32(0))
        got = med3(p, q, b2)
        old = med3(p, q, np.copysign(np.float32(np.inf), b))
        finite = np.isfinite(b2) & np.isfinite(a + a)
    assert np.array_equal(got[finite], old[finite])
    want = superbee_def(a, b)
    # +0 and -0 compare equal; the definition's sign test is exact here (no product underflow)
    assert np.array_equal(got[finite], want[finite])
