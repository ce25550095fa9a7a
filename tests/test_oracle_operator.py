"""Pins of the oracle's viscous matrix A(dt) against properties the paper and
linear algebra fix: row sums, diagonal dominance, symmetry conditions,
positive spectrum, the continuum Laplacian and the harmonic-mean limit."""
import numpy as np
import pytest

import oracle as O
from paper_2206_14780_amd import workloads as W


def _tank(seed=7, n=(6, 6, 5), wall=W.WALL_DUMMY, avg=W.AVG_HARMONIC, mu_span=100.0,
          dt_nu=10.0, jitter=0.2, uniform=False):
    """Small jittered fluid block in a periodic x-y channel with three wall
    layers at top and bottom; viscosity log-uniform over mu_span."""
    rng = np.random.default_rng(seed)
    pos, pt = W.lattice(n, 1.0, walls=((False, False), (False, False), (True, True)),
                        jitter=jitter, rng=rng)
    N = pos.shape[0]
    if uniform:
        mu = np.ones(N)
        mass = np.ones(N)
        rho = np.ones(N)
    else:
        mu = 10.0 ** rng.uniform(0.0, np.log10(mu_span), N)
        rho = rng.uniform(0.95, 1.05, N)
        mass = rho * rng.uniform(0.97, 1.03, N)
    period = np.array([n[0], n[1], 0.0])
    dt = dt_nu / mu.max()
    return dict(pos=pos, mass=mass, rho=rho, mu=mu, ptype=pt, period=period, h=1.3, dt=dt,
                wall=wall, avg=avg), pt


@pytest.mark.parametrize("wall", [W.WALL_DYNAMIC, W.WALL_DUMMY])
@pytest.mark.parametrize("avg", [W.AVG_ARITH, W.AVG_HARMONIC])
def test_row_sums(wall, avg):
    # eqs. diag/offdiag: each fluid row sums to 1 (1 + dt sum w - dt sum w);
    # dynamic wall rows are identity; a dummy wall row sums to 2 when it has
    # fluid neighbours (1 + sum W / sum W, eq. implicit-system-dummy-full).
    kw, pt = _tank(wall=wall, avg=avg)
    op = O.Operator(jacobi=False, **kw)
    y = op.apply(np.ones((pt.size, 3)))
    fl = pt == W.FLUID
    assert np.allclose(y[fl], 1.0, rtol=0, atol=1e-12)
    if wall == W.WALL_DYNAMIC:
        assert np.all(y[~fl] == 1.0)
    else:
        rp, cols = op.row_ptr, op.cols
        has_fluid = np.array([np.any(pt[cols[rp[i]:rp[i + 1]]] == W.FLUID) for i in range(pt.size)])
        assert np.allclose(y[~fl & has_fluid], 2.0, atol=1e-13)
        assert np.all(y[~fl & ~has_fluid] == 1.0)
        assert np.any(~fl & ~has_fluid)  # the third wall layer is beyond 2h of the fluid


@pytest.mark.parametrize("jacobi", [False, True])
@pytest.mark.parametrize("wall", [W.WALL_DYNAMIC, W.WALL_DUMMY])
def test_dense_assembly_matches_matrix_free(jacobi, wall):
    kw, pt = _tank(wall=wall)
    op = O.Operator(jacobi=jacobi, **kw)
    A = op.dense()
    X = np.random.default_rng(0).normal(size=(pt.size, 3))
    assert np.allclose(A @ X, op.apply(X), rtol=1e-13, atol=1e-13)
    if jacobi:
        assert np.allclose(np.diag(A), 1.0)
    else:
        assert np.allclose(np.diag(A), op.diag(), rtol=1e-15)


def test_diagonal_dominance():
    # Fluid rows are strictly diagonally dominant; dummy-wall rows are only
    # weakly dominant but every off-diagonal entry points at an SDD fluid row
    # (weakly chained diagonally dominant => non-singular).
    kw, pt = _tank(wall=W.WALL_DUMMY)
    A = O.Operator(jacobi=False, **kw).dense()
    off = np.abs(A).sum(axis=1) - np.abs(np.diag(A))
    fl = pt == W.FLUID
    assert np.all(np.abs(np.diag(A))[fl] > off[fl])
    assert np.all(np.abs(np.diag(A))[~fl] >= off[~fl] - 1e-12)
    for i in np.where(~fl)[0]:
        nz = np.nonzero(A[i])[0]
        assert np.all(fl[nz[nz != i]])
    assert np.linalg.matrix_rank(A) == A.shape[0]


@pytest.mark.parametrize("avg", [W.AVG_ARITH, W.AVG_HARMONIC])
def test_fluid_block_symmetric_bitwise(avg):
    # Symmetric when masses and densities are uniform and the mean viscosity
    # is symmetric (Section "Linear system properties", appendix on symmetry
    # pitfalls) -- bitwise, since contraction is off and r_ab = -r_ba exactly.
    kw, pt = _tank(wall=W.WALL_DYNAMIC, avg=avg, uniform=True)
    kw["mu"] = 10.0 ** np.random.default_rng(3).uniform(0, 2, pt.size)
    A = O.Operator(jacobi=False, **kw).dense()
    fl = np.where(pt == W.FLUID)[0]
    Aff = A[np.ix_(fl, fl)]
    assert np.array_equal(Aff, Aff.T)
    # A = I + dt L with L positive semi-definite: every eigenvalue >= 1
    # (the diffusive sign reading of eq. kab; the printed sign would give
    # eigenvalues below 1 and indefinite matrices).
    assert np.linalg.eigvalsh(Aff).min() >= 1.0 - 1e-10


def test_dummy_walls_break_symmetry():
    kw, pt = _tank(wall=W.WALL_DUMMY, uniform=True)
    A = O.Operator(jacobi=False, **kw).dense()
    assert np.abs(A - A.T).max() > 1e-3


def test_operator_approximates_viscous_laplacian():
    # (u - A u)/dt = sum_a w_ba (u_a - u_b) approximates nu lap(u) (eq.
    # part_NS viscous term).  On a periodic lattice with h = 1.3 dp the Wendland
    # sum underestimates the Laplacian by a few per cent, the same bias that
    # makes the Poiseuille profile ~2 % high in the paper.
    n, nz = 8, 32
    pos, pt = W.lattice((n, n, nz), 1.0)
    op = O.Operator(pos, 1.0, 1.0, 2.5, pt, [n, n, nz], 1.3, 0.7, 0, 0, jacobi=False)
    k = 2 * np.pi / nz
    u = np.zeros((pos.shape[0], 3))
    u[:, 1] = np.sin(k * pos[:, 2])
    lap = (u - op.apply(u)) / 0.7
    sel = np.abs(u[:, 1]) > 0.5
    ratio = lap[sel, 1] / (-2.5 * k * k * u[sel, 1])
    assert np.all(np.abs(ratio - 0.975) < 0.01)


def test_harmonic_mean_limit():
    # Harmonic mean of mu_b and mu_a -> infinity tends to 2 mu_b, so a fluid
    # row whose neighbours are all very viscous equals, under harmonic
    # averaging, the arithmetic-average row of a fluid with viscosity 2 mu_b.
    kw, pt = _tank(wall=W.WALL_DYNAMIC, uniform=True)
    N = pt.size
    i0 = np.where(pt == W.FLUID)[0][len(np.where(pt == W.FLUID)[0]) // 2]
    mu_h = np.full(N, 1e13)
    mu_h[i0] = 0.8
    mu_a = np.full(N, 1.6)
    X = np.random.default_rng(1).normal(size=(N, 3))
    kw_h = dict(kw, mu=mu_h, avg=W.AVG_HARMONIC, dt=0.3)
    kw_a = dict(kw, mu=mu_a, avg=W.AVG_ARITH, dt=0.3)
    yh = O.Operator(jacobi=False, **kw_h).apply(X)[i0]
    ya = O.Operator(jacobi=False, **kw_a).apply(X)[i0]
    assert np.allclose(yh, ya, rtol=1e-9)


@pytest.mark.parametrize("wall", [W.WALL_DYNAMIC, W.WALL_DUMMY])
@pytest.mark.parametrize("jacobi", [True, False])
def test_assembled_entries_equal_the_dense_assembly(wall, jacobi):
    # The stored sparse entries are the dense assembly's entries on the
    # neighbour pattern, bit for bit, and zero off it; multiplying by them
    # gives the matrix-free apply up to the rounding of a sum of ~80 terms.
    kw, pt = _tank(wall=wall, mu_span=1000.0, dt_nu=50.0)
    op = O.Operator(jacobi=jacobi, **kw)
    A = op.dense()
    d, e = op.entries()
    n = pt.size
    rows = np.repeat(np.arange(n), np.diff(op.row_ptr))
    S = np.zeros((n, n))
    S[np.arange(n), np.arange(n)] = d
    S[rows, op.cols] += e
    assert np.array_equal(S, A)
    X = np.random.default_rng(3).normal(size=(n, 3))
    Y = op.apply(X)
    Ya = O.Operator(jacobi=jacobi, **kw).assemble().apply(X)
    scale = (np.abs(A) @ np.abs(X)).max()
    assert np.max(np.abs(Ya - Y)) <= 200 * 2.0 ** -53 * scale
    assert np.max(np.abs(Ya - A @ X)) <= 200 * 2.0 ** -53 * scale
    # and a solve on the assembled operator reaches the same answer
    B = np.random.default_rng(4).normal(size=(n, 3))
    Xs, rep, _ = O.solve(O.Operator(jacobi=jacobi, **kw).assemble(), B, tol=1e-13)
    Xd = O.dense_solve(op, B)
    assert rep["status"] == 0 and np.linalg.norm(Xs - Xd) / np.linalg.norm(Xd) < 1e-10
