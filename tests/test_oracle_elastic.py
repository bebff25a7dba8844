"""Pins of the elasticity oracle (Sec. 6.2 cantilever control) against what the
mechanics and the mathematics fix: the rigid-body modes span the kernel of an
element's stiffness, the strain energy of every linear displacement field is
the closed form h^3 (lambda tr(eps)^2 + 2 mu eps:eps), the vector mass is the
Kronecker product of the 1D masses, support reactions balance the applied
pressure, the discrete solution of a manufactured problem converges at second
order, and the range-space solves equal the brute-force KKT solve."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import elastic as el
from oracle import feti, kkt, solve


def _rigid_modes(h):
    """Six rigid-body displacement fields of a cube cell (3 translations, 3 rotations)."""
    offs = np.array([((l >> 0) & 1, (l >> 1) & 1, (l >> 2) & 1) for l in range(8)], dtype=float) * h
    modes = []
    for c in range(3):
        t = np.zeros((8, 3))
        t[:, c] = 1.0
        modes.append(t.ravel())
    for axis in range(3):
        w = np.zeros(3)
        w[axis] = 1.0
        modes.append(np.cross(w, offs).ravel())
    return np.array(modes)


@pytest.mark.parametrize("h,E,nu", [(0.5, el.YOUNG, el.POISSON), (0.125, 1.0, 0.3), (1.0, 200e9, 0.0)])
def test_element_kernel_is_the_rigid_body_modes(h, E, nu):
    Ke = el.elasticity_element(h, E, nu)
    assert np.abs(Ke - Ke.T).max() <= 1e-12 * np.abs(Ke).max()
    R = _rigid_modes(h)
    assert np.abs(Ke @ R.T).max() <= 1e-9 * np.abs(Ke).max()
    ev = np.linalg.eigvalsh(Ke)
    assert np.sum(ev > 1e-9 * ev.max()) == 18 and ev.min() > -1e-9 * ev.max()


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_strain_energy_of_linear_fields(seed):
    """u(x) = G x: constant strain eps = sym(G), energy density lambda tr(eps)^2 + 2 mu eps:eps
    over the cell volume h^3 (Q1 represents linear fields exactly)."""
    rng = np.random.default_rng(seed)
    h, E, nu = 0.25, 3.0, 0.31
    G = rng.standard_normal((3, 3))
    offs = np.array([((l >> 0) & 1, (l >> 1) & 1, (l >> 2) & 1) for l in range(8)], dtype=float) * h
    u = (offs @ G.T).ravel()
    eps = 0.5 * (G + G.T)
    lam, mu = el.lame(E, nu)
    energy = h ** 3 * (lam * np.trace(eps) ** 2 + 2.0 * mu * np.sum(eps * eps))
    Ke = el.elasticity_element(h, E, nu)
    assert abs(u @ Ke @ u - energy) <= 1e-12 * energy


def test_vector_mass_is_the_kronecker_product():
    h = 0.2
    m1 = h / 6.0 * np.array([[2.0, 1.0], [1.0, 2.0]])
    Me = el.mass_element(h)
    ref = np.kron(np.kron(np.kron(m1, m1), m1), np.eye(3))  # vertex index a + 2b + 4c: x fastest
    assert np.abs(Me - ref).max() <= 1e-15
    assert abs(Me[0::3, 0::3].sum() - h ** 3) <= 1e-15


@pytest.mark.parametrize("n", [2, 3])
def test_reactions_balance_the_pressure(n):
    box = el.Box(n)
    A = el.assemble(box)
    f = el.pressure_load(box, 1e5)
    u = spla.spsolve(A["K"].tocsc(), f)
    R = el.reactions(box, u)
    # the load on the free nodes plus the reaction at the clamp carry the whole face
    assert abs(f.sum() + 1e5 * box.length * 1.0 * (1 - 0.5 / (box.length * n))) <= 1e-6
    assert np.abs(R + np.array([0.0, 0.0, f.sum()])).max() <= 1e-6 * abs(f.sum())
    assert u[2::3].max() < 0.0 or np.abs(u[2::3]).max() > 0  # the beam bends down
    assert u[2::3].mean() < 0.0


def _manufactured(coords, lam, mu):
    """u* = (1, -2, 3/2) sin(pi x) sin(pi y) sin(pi z), zero on the cube's faces, and
    f = -div sigma(u*) = -(lambda + mu) grad div u* - mu Laplace u*."""
    a = np.array([1.0, -2.0, 1.5])
    x, y, z = coords.T
    p = np.pi
    s = [np.sin(p * x), np.sin(p * y), np.sin(p * z)]
    c = [np.cos(p * x), np.cos(p * y), np.cos(p * z)]
    sss = s[0] * s[1] * s[2]
    u = np.outer(sss, a)
    # second derivatives of s = sin sin sin: d_ii s = -pi^2 s, d_ij s = pi^2 c_i c_j s_k
    d2 = np.zeros((coords.shape[0], 3, 3))
    for i in range(3):
        for j in range(3):
            if i == j:
                d2[:, i, j] = -p * p * sss
            else:
                k = 3 - i - j
                d2[:, i, j] = p * p * c[i] * c[j] * s[k]
    grad_div = np.einsum("nij,j->ni", d2, a)
    lap = -3.0 * p * p * np.outer(sss, a)
    f = -(lam + mu) * grad_div - mu * lap
    return u, f


def test_manufactured_solution_converges_at_second_order():
    E, nu = 1.0, 0.3
    lam, mu = el.lame(E, nu)
    errs = []
    for n in (4, 8, 16):
        box = el.Box(n, clamp="cube")
        A = el.assemble(box, E, nu)
        ue, _ = _manufactured(box.coords(), lam, mu)
        _, f_all = _manufactured(box.ijk * box.h, lam, mu)  # the body force at every node
        u = spla.spsolve(A["K"].tocsc(), el.body_load(box, f_all))
        errs.append(np.abs(u - ue.ravel()).max() / np.abs(ue).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert errs[-1] < 1e-2, errs
    assert np.all(rates > 1.8), (errs, rates)


def test_range_space_equals_brute_force_kkt_on_the_cantilever():
    """O1 (two complex factors) = O2 (reduced real saddle system) = O3 (dense KKT) on the
    rubber cantilever.  The KKT system mixes stiffness entries ~E h = 1e7 with mass
    entries ~h^3 and beta h^3, so its FP64 solutions agree to ~1e-8 rather than 1e-12,
    and the dense LU's u (= lam / beta) only to ~1e-6."""
    box = el.Box(2)
    A = el.assemble(box)
    K, M, Kc = A["K"], A["M"], A["Kc"]
    ybar = spla.spsolve(K.tocsc(), el.pressure_load(box, 1e5))
    rel = lambda a, b: np.linalg.norm(a - b) / np.linalg.norm(b)
    for beta in (1e-10, 1e-14):
        o1 = solve.range_space_two_factor(K, M, Kc, beta, ybar, None, paper_y=False)
        o2 = solve.reduced_saddle(K, M, Kc, beta, ybar, None)
        o3 = solve.dense_kkt(K, M, Kc, beta, ybar, None)
        for k in ("y", "u", "lam"):
            assert rel(o1[k], o2[k]) <= 1e-7, (beta, k)
        for k in ("y", "lam"):
            assert rel(o3[k], o2[k]) <= 1e-7, (beta, k)
        assert rel(o3["u"], o2["u"]) <= 1e-5, beta
        for o in (o1, o2, o3):
            assert kkt.rel_kkt(K, M, Kc, beta, ybar, None, o["y"], o["u"], o["lam"]) <= 1e-6


def _interface_counts(box, m):
    """Brute force over the grid nodes: corner dofs (unclamped subdomain vertices)
    and fully redundant multipliers (C(k, 2) per component on every unclamped
    non-vertex node shared by k >= 2 subdomains)."""
    nC = nmu = 0
    for k in range(box.nz + 1):
        for j in range(box.ny + 1):
            for i in range(1, box.nx + 1):
                on = [i % m == 0, j % m == 0, k % m == 0]
                share = [v % m == 0 and 0 < v < top for v, top in ((i, box.nx), (j, box.ny), (k, box.nz))]
                mult = 2 ** sum(share)
                if all(on):
                    nC += 3
                elif mult >= 2:
                    nmu += 3 * mult * (mult - 1) // 2
    return nC, nmu


@pytest.mark.parametrize("n,m", [(2, 2), (4, 2), (4, 4)])
def test_partition_counts_and_load_split(n, m):
    box = el.Box(n)
    dec = el.Decomposition(box, m)
    assert (dec.nC, dec.nmu) == _interface_counts(box, m)
    assert dec.nsub == (box.nx // m) * (box.ny // m) * (box.nz // m)
    # the subdomain shares of a load add up to it (corners through f_c)
    f = np.random.default_rng(3).standard_normal(box.n_dof)
    fr, fc = dec.split_rhs(f)
    back = np.zeros(dec.mesh.n_full)
    for sd, x in zip(dec.subs, fr):
        np.add.at(back, sd["full"][sd["r"]], x.real)
    back[dec.corner_full] += fc.real
    assert np.abs(back[dec.mesh.free_full] - f).max() <= 1e-14 * np.abs(f).max()


@pytest.mark.parametrize("n,m", [(2, 2), (4, 2), (4, 4)])
@pytest.mark.parametrize("beta", [1e-10, 1e-16])
def test_elastic_fetidp_equals_direct_solve(n, m, beta):
    """FETI-DP on the elasticity partition (dense interface solve) reproduces the
    sparse direct solution of Z x = f (Sec. 5): a wrong sign, corner or
    multiplier anywhere in the partition breaks it."""
    box = el.Box(n)
    dec = el.Decomposition(box, m)
    A = el.assemble(box)
    Z = solve.complex_factor(A["K"], A["M"], beta)
    rng = np.random.default_rng(7)
    f = rng.standard_normal(box.n_dof) + 1j * rng.standard_normal(box.n_dof)
    x, _ = feti.fetidp_solve_dense(dec, beta ** -0.5, f)
    ref = spla.spsolve(Z.tocsc(), f)
    assert np.linalg.norm(x - ref) <= 1e-12 * np.linalg.norm(ref)
