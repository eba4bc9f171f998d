"""The density kernel's float64 shortcut for the key bin, checked on the CPU.

For alpha = +1 the selection key is K = floor(U 2^31 / w).  The density
kernel stores only its 12-bit log-scale bin and takes it from the float64
value of x = U 2^31 / w, falling back to the exact quotient when x is below
256 or within 64 float64 steps of a bin edge.  This re-states that rule in
numpy (float64 with a correctly rounded 1/w, plus a deliberate relative
perturbation of up to 2^-50 standing for the hardware reciprocal's residual
error) and checks that whenever the rule claims the bin, the claim equals the
bin of the exact integer quotient, on random keys and on keys placed at and
next to every bin edge.
"""
import numpy as np

from gpu_util import kbin_of


def fast_bin(U, w, pert):
    x = U.astype(np.float64) * (1.0 / w.astype(np.float64)) * (1.0 + pert) * 2147483648.0
    bits = x.view(np.uint64)
    E = (bits >> np.uint64(52)).astype(np.int64) - 1023
    rest = bits & np.uint64((1 << 46) - 1)
    b = 128 + (E - 7) * 64 + ((bits >> np.uint64(46)) & np.uint64(63)).astype(np.int64)
    ok = (E >= 8) & (rest > np.uint64(64)) & (rest < np.uint64((1 << 46) - 64))
    return b, ok


def exact_bin(U, w):
    return kbin_of((U.astype(np.uint64) << np.uint64(31)) // w.astype(np.uint64))


def check(U, w, rng):
    for pert in (0.0, 2.0 ** -50, -(2.0 ** -50)):
        p = pert * rng.random(U.shape)
        b, ok = fast_bin(U, w, p)
        eb = exact_bin(U, w)
        assert np.array_equal(b[ok], eb[ok])
    return ok


def test_random_keys():
    rng = np.random.default_rng(5)
    n = 400_000
    U = rng.integers(1, 2 ** 32 + 1, n, dtype=np.uint64)
    w = np.concatenate([rng.integers(1, 64, n // 2), rng.integers(1, 2 ** 31, n - n // 2)]).astype(np.uint64)
    ok = check(U, w, rng)
    assert ok.mean() > 0.99      # the exact fallback is rare on random keys


def test_keys_at_bin_edges():
    # U 2^31 / w at, just below and just above integer bin edges: w = 2^k
    # makes x = U 2^(31-k) exact, so edges are hit exactly; odd w lands
    # within a fraction of a unit of them.
    rng = np.random.default_rng(6)
    Us, ws = [], []
    for k in range(0, 31):
        w = 1 << k
        for e in range(8, 63):
            for m in (64, 65, 100, 127, 128):
                edge = m << (e - 6)                   # a bin edge (128 << (e-6) is the next octave)
                for d in (-2, -1, 0, 1, 2):
                    num = (edge + d) * w             # U 2^31 = num (exactly when divisible)
                    if num % (1 << 31):
                        continue
                    U = num >> 31
                    if 1 <= U <= 2 ** 32:
                        Us.append(U); ws.append(w)
    for w in (3, 5, 7, 1000003, 2 ** 31 - 1):
        for e in range(8, 62):
            for m in (64, 96, 127):
                edge = m << (e - 6)
                U = (edge * w) >> 31
                for d in (-1, 0, 1, 2):
                    if 1 <= U + d <= 2 ** 32:
                        Us.append(U + d); ws.append(w)
    U = np.array(Us, dtype=np.uint64)
    w = np.array(ws, dtype=np.uint64)
    assert len(U) > 1000
    check(U, w, rng)
