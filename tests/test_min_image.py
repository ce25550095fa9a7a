"""The minimum-image displacement without a division.

Every neighbour test of the library takes the periodic displacement as
d - period * rint(d / period) (d = xb - xa), rounded the same way as the
oracle's, so that both decide the same pairs.  The device evaluates it
without the division for |d| < period: 0 correction for |d| <= period/2,
exactly +-period above.  This checks that branch structure bit for bit
against the formula with the division, on random differences and on the
doubles next to +-period/2, +-period and +-3 period/2 (ties included: a
quotient of exactly 1/2 rounds to 0), for periods that are and are not
powers of two.  The device code itself is checked by the GPU neighbour
tests, which include pairs at exactly half a period."""
import numpy as np


def _with_division(d, p):
    return d - p * np.rint(d / p)


def _branch_form(d, p):
    a = np.abs(d)
    out = d.copy()
    wrap = a > 0.5 * p
    near = wrap & (a < p)
    out[near] = d[near] - np.copysign(p, d[near])
    far = wrap & ~(a < p)
    out[far] = d[far] - p * np.rint(d[far] / p)
    return out


def _boundary_values(p, ulps=40):
    vals = []
    for c in (0.5, 1.0, 1.5):
        for s in (1.0, -1.0):
            x = s * c * p
            up = down = x
            for _ in range(ulps):
                vals += [up, down]
                up, down = np.nextafter(up, np.inf), np.nextafter(down, -np.inf)
    return np.array(vals)


def test_branch_form_equals_division_form_bitwise():
    rng = np.random.default_rng(11)
    for p in (1.0, 4.0, 320.0, 3.0, 0.1, 1.0 / 3.0, 100.7, 0.21875, 1e6 + 0.3):
        xa, xb = rng.uniform(0.0, p, 20000), rng.uniform(0.0, p, 20000)
        d = np.concatenate([xb - xa, rng.uniform(-2.0 * p, 2.0 * p, 20000), _boundary_values(p)])
        ref, got = _with_division(d, p), _branch_form(d, p)
        assert np.array_equal(ref.view(np.int64), got.view(np.int64)), p


def test_tie_and_next_doubles():
    # half a period exactly: rint(1/2) = 0, no wrap; one ulp above: wrap
    p = 3.0
    assert _branch_form(np.array([1.5]), p)[0] == 1.5
    assert _branch_form(np.array([-1.5]), p)[0] == -1.5
    up = np.nextafter(1.5, 2.0)
    assert _branch_form(np.array([up]), p)[0] == up - 3.0 == _with_division(np.array([up]), p)[0]
