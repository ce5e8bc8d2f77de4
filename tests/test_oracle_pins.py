"""Pins of the CPU oracle against what the mathematics fixes.

Nothing here retypes the oracle's recurrences: every expected value comes
from a closed form evaluated with mpmath / scipy, a derivative identity of
that closed form, brute-force quadrature, a brute-force n^4 contraction, an
invariant, or a count printed in the paper.
"""

import math
import os

import mpmath as mp
import numpy as np
import pytest
from scipy import special

import hfx_inputs as hi
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- Boys ----
def _boys_mp(m, T):
    # F_m(T) = 1F1(m+1/2; m+3/2; -T) / (2m+1)
    return mp.hyp1f1(m + mp.mpf(1) / 2, m + mp.mpf(3) / 2, -mp.mpf(T)) / (2 * m + 1)


@pytest.mark.parametrize("m", [0, 1, 2, 4, 8, 12])
@pytest.mark.parametrize("T", [0.0, 1e-9, 0.3, 2.5, 11.0, 29.999, 30.0, 30.001, 44.0, 120.0, 900.0])
def test_boys_vs_mpmath(m, T):
    mp.mp.dps = 40
    ref = float(_boys_mp(m, T))
    got = oracle.boys(m, T)
    assert abs(got - ref) <= 2e-15 * abs(ref) + 1e-300


@pytest.mark.parametrize("T", [1e-6, 0.7, 5.0, 31.0, 80.0])
def test_boys_F0_closed_form_and_gammainc(T):
    f0 = math.sqrt(math.pi) * math.erf(math.sqrt(T)) / (2 * math.sqrt(T))
    assert abs(oracle.boys(0, T) - f0) < 1e-15
    for m in range(6):
        ref = special.gamma(m + 0.5) * special.gammainc(m + 0.5, T) / (2 * T ** (m + 0.5))
        assert abs(oracle.boys(m, T) - ref) <= 1e-13 * ref


def test_boys_zero_and_downward_identity():
    for m in range(10):
        assert oracle.boys(m, 0.0) == pytest.approx(1.0 / (2 * m + 1), rel=1e-16, abs=0)
    for T in (0.1, 3.0, 17.0, 35.0):
        for m in range(8):
            lhs = oracle.boys(m, T)
            rhs = (2 * T * oracle.boys(m + 1, T) + math.exp(-T)) / (2 * m + 1)
            assert abs(lhs - rhs) <= 4e-15 * lhs


# ------------------------------------------------------- basis helpers ----
def _one_shell_sys(centres, ls, exps, coefs=None, P=None):
    shells = []
    for a, (l, e) in enumerate(zip(ls, exps)):
        e = np.atleast_1d(np.asarray(e, dtype=float))
        c = np.ones_like(e) if coefs is None else np.atleast_1d(coefs[a])
        shells.append((a, l, e, c))
    nbf = sum(2 * l + 1 for l in ls)
    return hi._pack(np.asarray(centres, dtype=float), shells,
                    np.eye(nbf) if P is None else P, dict(name="pin"))


def _ssss_closed_mp(a, A, b, B, c, C, d, D, omega=0):
    """Unnormalised primitive (ss|ss) (Gaussian charge distributions), mpmath."""
    A, B, C, D = [[mp.mpf(x) for x in v] for v in (A, B, C, D)]
    a, b, c, d = mp.mpf(a), mp.mpf(b), mp.mpf(c), mp.mpf(d)
    p, q = a + b, c + d
    P = [(a * A[i] + b * B[i]) / p for i in range(3)]
    Q = [(c * C[i] + d * D[i]) / q for i in range(3)]
    ab2 = sum((A[i] - B[i]) ** 2 for i in range(3))
    cd2 = sum((C[i] - D[i]) ** 2 for i in range(3))
    pq2 = sum((P[i] - Q[i]) ** 2 for i in range(3))
    rho = p * q / (p + q)

    def F0(T):
        return mp.mpf(1) if T == 0 else mp.sqrt(mp.pi) * mp.erf(mp.sqrt(T)) / (2 * mp.sqrt(T))

    T = rho * pq2
    g = F0(T)
    if omega:
        w = mp.mpf(omega)
        th2 = w * w / (w * w + rho)
        g -= mp.sqrt(th2) * F0(th2 * T)
    return 2 * mp.pi ** mp.mpf(2.5) / (p * q * mp.sqrt(p + q)) * mp.exp(-a * b / p * ab2 - c * d / q * cd2) * g


def _norm_prim(alpha, l):
    return (2 * alpha / math.pi) ** 0.75 * (4 * alpha) ** (l / 2) / math.sqrt(
        [1, 1, 3][l])


def test_golden_one_centre_ssss():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "one_centre_ssss.txt")) if l.strip() and not l.startswith("#")]
    s = _one_shell_sys([[0, 0, 0]], [0], [[1.0]])
    for om, val in rows:
        got = oracle.shell_quartet(s, 0, 0, 0, 0, omega=float(om))[0, 0, 0, 0]
        assert abs(got - float(val)) < 1e-15


@pytest.mark.parametrize("omega", [0.0, 0.11, 0.7])
def test_contracted_ssss_closed_form(omega):
    rng = np.random.default_rng(7)
    cen = rng.uniform(-2, 2, size=(4, 3))
    exps = [rng.uniform(0.1, 5, size=3) for _ in range(4)]
    coefs = [rng.uniform(0.1, 1, size=3) for _ in range(4)]
    s = _one_shell_sys(cen, [0, 0, 0, 0], exps, coefs)
    cn = oracle.normalised_coefs(s)
    mp.mp.dps = 30
    ref = mp.mpf(0)
    for i in range(3):
        for j in range(3):
            for k in range(3):
                for l in range(3):
                    w = cn[i] * cn[3 + j] * cn[6 + k] * cn[9 + l]
                    ref += w * _ssss_closed_mp(exps[0][i], cen[0], exps[1][j], cen[1],
                                               exps[2][k], cen[2], exps[3][l], cen[3], omega)
    got = oracle.shell_quartet(s, 0, 1, 2, 3, omega=omega)[0, 0, 0, 0]
    assert abs(got - float(ref)) <= 1e-14 * abs(float(ref))


def test_normalisation_unit_overlap():
    """One-centre overlap of each normalised contracted shell is the identity
    (spherical): checked with the closed Gaussian overlap integral."""
    rng = np.random.default_rng(3)
    for l in (0, 1, 2):
        e = rng.uniform(0.1, 8, size=4)
        c = rng.uniform(0.1, 1, size=4)
        s = _one_shell_sys([[0, 0, 0]], [l], [e], [c])
        cn = oracle.normalised_coefs(s)
        # <x^l g_p | x^l g_q> for the x^l component with primitive norms folded in:
        # int x^(2l) exp(-(a+b) r^2) = (2l-1)!!/(2(a+b))^l (pi/(a+b))^(3/2)
        S = 0.0
        for p in range(4):
            for q in range(4):
                ab = e[p] + e[q]
                S += cn[p] * cn[q] * [1, 1, 3][l] / (2 * ab) ** l * (math.pi / ab) ** 1.5
        assert abs(S - 1.0) < 1e-13
        # primitive factor of a single-primitive shell equals the textbook one
        s1 = _one_shell_sys([[0, 0, 0]], [l], [[e[0]]], [[0.37]])
        assert abs(oracle.normalised_coefs(s1)[0] - _norm_prim(e[0], l)) < 1e-13 * _norm_prim(e[0], l)


# ------------------------------------ p and d via derivative identities ----
# x_A^k g(A) relates to derivatives of the s Gaussian with respect to A:
#   x_A g = (1/2a) dg/dA_x,   x_A y_A g = (1/4a^2) d2g/dA_x dA_y,
#   x_A^2 g = (1/4a^2) (d2/dA_x^2 + 2a) g.
# Spherical d from Cartesians normalised like x^2 (Sec. 3 transformation):
#   xy, yz, z2 - (x2 + y2)/2, xz, (x2 - y2) sqrt(3)/2   with sqrt3 on xy, yz, xz.
_R3 = math.sqrt(3.0)
_SPH = {
    0: [[((0, 0, 0), 1.0)]],
    1: [[((1, 0, 0), 1.0)], [((0, 1, 0), 1.0)], [((0, 0, 1), 1.0)]],
    2: [[((1, 1, 0), _R3)], [((0, 1, 1), _R3)],
        [((0, 0, 2), 1.0), ((2, 0, 0), -0.5), ((0, 2, 0), -0.5)],
        [((1, 0, 1), _R3)], [((2, 0, 0), 0.5 * _R3), ((0, 2, 0), -0.5 * _R3)]],
}


def _cart_from_derivs(f, exps, pows, x0):
    """Unnormalised primitive Cartesian integral for monomial powers `pows`
    (one (i,j,k) per centre) from derivatives of the s closed form f(x12)."""
    # Each centre contributes a linear operator in its 3 coordinates;
    # expand x^2 terms into (d2 + 2a) and collect derivative multi-indices.
    terms = [((0,) * 12, mp.mpf(1))]
    for ci, (pw, a) in enumerate(zip(pows, exps)):
        a = mp.mpf(a)
        new = []
        for t, w in terms:
            opts = [([0, 0, 0], mp.mpf(1))]
            for ax in range(3):
                k = pw[ax]
                if k == 0:
                    continue
                if k == 1:
                    opts = [(o[:ax] + [o[ax] + 1] + o[ax + 1:], wo / (2 * a)) for o, wo in opts]
                else:  # k == 2
                    o2 = []
                    for o, wo in opts:
                        o2.append((o[:ax] + [o[ax] + 2] + o[ax + 1:], wo / (4 * a * a)))
                        o2.append((o, wo * 2 * a / (4 * a * a)))
                    opts = o2
            for o, wo in opts:
                tt = list(t)
                for ax in range(3):
                    tt[3 * ci + ax] += o[ax]
                new.append((tuple(tt), w * wo))
        terms = new
    tot = mp.mpf(0)
    for t, w in terms:
        if sum(t) == 0:
            tot += w * f(*x0)
        else:
            tot += w * mp.diff(f, x0, t)
    return tot


@pytest.mark.parametrize("ls", [(1, 0, 0, 0), (1, 1, 0, 0), (1, 0, 1, 0), (1, 1, 1, 1), (2, 0, 0, 0),
                                (2, 1, 0, 0), (2, 0, 2, 0), (2, 1, 1, 0), (2, 2, 0, 0), (2, 1, 2, 1),
                                (2, 2, 2, 1), pytest.param((2, 2, 2, 2), marks=pytest.mark.slow), (0, 2, 1, 0)])
@pytest.mark.parametrize("omega", [0.0, 0.11])
def test_p_d_against_derivatives_of_closed_form(ls, omega):
    """Single-primitive shells: selected spherical components vs derivatives
    of the mpmath closed-form (ss|ss) with respect to the centres.  The (dd|dd)
    case (an eighth-order derivative, minutes) runs with HFX_SLOW=1; in the
    default suite (dd|dd) is pinned by the McMurchie-Davidson evaluation."""
    rng = np.random.default_rng(hash(ls) % 1000 + int(omega * 100))
    cen = rng.uniform(-1.2, 1.2, size=(4, 3))
    ex = rng.uniform(0.3, 2.0, size=4)
    s = _one_shell_sys(cen, list(ls), [[e] for e in ex])
    got = oracle.shell_quartet(s, 0, 1, 2, 3, omega=omega)
    # the derivative order is the total L; at L >= 7 one component at a lower
    # working precision keeps the run to seconds (mpmath raises the precision
    # of its difference quotients by itself)
    mp.mp.dps = 24 if sum(ls) < 7 else 16
    x0 = [mp.mpf(float(v)) for v in cen.ravel()]

    def f(*x):
        return _ssss_closed_mp(ex[0], x[0:3], ex[1], x[3:6], ex[2], x[6:9], ex[3], x[9:12], omega)

    norms = [_norm_prim(ex[i], ls[i]) for i in range(4)]
    shape = got.shape
    if sum(ls) <= 4:
        picks = [tuple(int(rng.integers(0, n)) for n in shape) for _ in range(3)]
    else:  # single-monomial components keep the high-order derivatives cheap
        one = {0: [0], 1: [0, 1, 2], 2: [0, 1, 3]}
        picks = [tuple(int(rng.choice(one[l])) for l in ls) for _ in range(2 if sum(ls) < 7 else 1)]
    for idx in picks:
        ref = mp.mpf(0)
        combos = [[]]
        for ci in range(4):
            combos = [c + [t] for c in combos for t in _SPH[ls[ci]][idx[ci]]]
        for combo in combos:
            pows = [t[0] for t in combo]
            w = np.prod([t[1] for t in combo])
            ref += w * _cart_from_derivs(f, ex, pows, x0)
        ref *= np.prod(norms)
        assert abs(got[idx] - float(ref)) <= 1e-11 * max(1.0, abs(float(ref))), (idx, got[idx], float(ref))


# -------------------------------------------- brute-force quadrature ----
def _quad_s_only(sys, I, J, K, L, omega=0.0, nu=160, cn=None):
    """(IJ|KL) for s or p shells by brute force: the kernel written as a
    Gaussian transform, g(r) = 2/sqrt(pi) int_{omega}^inf exp(-u^2 r^2) du,
    the six-dimensional space integral factorised per Cartesian axis and each
    axis done on a trapezoid grid in (x, s = x - x'), u by Gauss-Legendre
    after u = omega + t/(1-t).  Uses only the Gaussian primitives' values."""
    cn = oracle.normalised_coefs(sys) if cn is None else cn
    sh = [I, J, K, L]
    tg, wg = np.polynomial.legendre.leggauss(nu)
    t = 0.5 * (tg + 1)
    w_t = 0.5 * wg
    u = omega + t / (1 - t)
    du = w_t / (1 - t) ** 2
    comps = []  # list over spherical components of per-shell (pows, weight)
    for s in sh:
        assert sys.shell_l[s] <= 1
    out_shape = tuple(int(2 * sys.shell_l[s] + 1) for s in sh)
    res = np.zeros(out_shape)
    prims = [[(sys.exps[sys.shell_off[s] + p], cn[sys.shell_off[s] + p]) for p in range(sys.shell_nprim[s])] for s in sh]
    cen = [sys.xyz[sys.shell_atom[s]] for s in sh]
    for idx in np.ndindex(*out_shape):
        pw = []
        for ci, s in enumerate(sh):
            p = [0, 0, 0]
            if sys.shell_l[s] == 1:
                p[idx[ci]] = 1
            pw.append(p)
        total = 0.0
        for pa in prims[0]:
            for pb in prims[1]:
                for pc in prims[2]:
                    for pd in prims[3]:
                        coef = pa[1] * pb[1] * pc[1] * pd[1]
                        J_u = np.ones_like(u)
                        for ax in range(3):
                            J_u *= _axis_integral(pa[0], cen[0][ax], pw[0][ax], pb[0], cen[1][ax], pw[1][ax],
                                                  pc[0], cen[2][ax], pw[2][ax], pd[0], cen[3][ax], pw[3][ax], u)
                        total += coef * np.sum(J_u * du)
        res[idx] = 2 / math.sqrt(math.pi) * total
    return res


def _axis_integral(a, A, ka, b, B, kb, c, C, kc, d, D, kd, u):
    zeta, eta = a + b, c + d
    Px, Qx = (a * A + b * B) / zeta, (c * C + d * D) / eta
    hx = 0.3 / math.sqrt(zeta)
    x = Px + hx * np.arange(-70, 71)
    gab = (x - A) ** ka * (x - B) ** kb * np.exp(-a * (x - A) ** 2 - b * (x - B) ** 2)
    k = np.arange(-45, 46)
    out = np.empty_like(u)
    for iu, uu in enumerate(u):
        if uu >= math.sqrt(eta):
            s = (0.3 / uu) * k[None, :] + 0.0 * x[:, None]     # kernel-centred samples
            hs = 0.3 / uu
        else:
            hs = 0.3 / math.sqrt(eta)
            s = (x - Qx)[:, None] + hs * k[None, :]            # ket-centred samples
        xp = x[:, None] - s
        gcd = (xp - C) ** kc * (xp - D) ** kd * np.exp(-c * (xp - C) ** 2 - d * (xp - D) ** 2)
        acc = hs * np.sum(gcd * np.exp(-(uu * s) ** 2), axis=1)
        out[iu] = hx * np.sum(gab * acc)
    return out


@pytest.mark.parametrize("omega", [0.0, 0.11])
def test_s_only_grid_quadrature(omega):
    """Tiny s-only input: every shell quartet of a 3-atom, 2-primitive s
    system against brute-force quadrature."""
    rng = np.random.default_rng(11)
    cen = rng.uniform(0, 3, size=(3, 3))
    exps = [rng.uniform(0.2, 3, size=2) for _ in range(3)]
    coefs = [rng.uniform(0.1, 1, size=2) for _ in range(3)]
    s = _one_shell_sys(cen, [0, 0, 0], exps, coefs)
    cn = oracle.normalised_coefs(s)
    for q in [(0, 0, 0, 0), (0, 1, 2, 2), (1, 2, 0, 1), (2, 1, 2, 0)]:
        ref = _quad_s_only(s, *q, omega=omega, cn=cn)
        got = oracle.shell_quartet(s, *q, omega=omega)
        assert np.allclose(got, ref, rtol=2e-11, atol=1e-13), (q, got.ravel(), ref.ravel())


def test_p_grid_quadrature():
    rng = np.random.default_rng(12)
    cen = rng.uniform(0, 2.5, size=(2, 3))
    s = _one_shell_sys(cen, [1, 0], [[0.9], [0.6]])
    ref = _quad_s_only(s, 0, 1, 0, 1, omega=0.11)
    got = oracle.shell_quartet(s, 0, 1, 0, 1, omega=0.11)
    assert np.allclose(got, ref, rtol=2e-11, atol=1e-13)


# ----------------------------------------------------------- invariants ----
@pytest.fixture(scope="module")
def small_spd():
    # s, p and d shells, 2 primitives, 3 atoms
    rng = np.random.default_rng(5)
    shells = []
    cen = rng.uniform(0, 4, size=(3, 3))
    for a in range(3):
        for l in (0, 1, 2):
            shells.append((a, l, rng.uniform(0.2, 4, size=2), rng.uniform(0.1, 1, size=2)))
    nbf = sum(2 * s[1] + 1 for s in shells)
    C = np.linalg.qr(rng.standard_normal((nbf, 6)))[0]
    return hi._pack(cen, shells, 2 * C @ C.T, dict(name="spd3"))


@pytest.mark.parametrize("omega", [0.0, 0.11])
def test_eight_fold_symmetry_schwarz_and_digestion(small_spd, omega):
    s = small_spd
    G = oracle.eri_tensor(s, omega=omega)
    for perm in [(1, 0, 2, 3), (0, 1, 3, 2), (2, 3, 0, 1), (3, 2, 1, 0), (2, 3, 1, 0)]:
        assert np.abs(G - G.transpose(perm)).max() <= 1e-14 * np.abs(G).max()
    D = np.einsum("ijij->ij", G)
    assert D.min() >= 0
    assert (np.abs(G) <= np.sqrt(np.einsum("ij,kl->ijkl", D, D)) * (1 + 1e-12) + 1e-14 * np.abs(G).max()).all()
    # ERI supermatrix positive semidefinite (positive kernel)
    n = s.nbf
    ev = np.linalg.eigvalsh(G.reshape(n * n, n * n))
    assert ev.min() > -1e-12 * ev.max()
    # unique-quartet digestion == brute-force n^4 contraction
    K, Q, cnt = oracle.build_K(s, tau=0.0, omega=omega)
    Kb = np.einsum("ijkl,jl->ik", G, s.P)
    assert np.abs(K - Kb).max() <= 1e-13 * np.abs(Kb).max()
    npair = s.nshell * (s.nshell + 1) // 2
    assert cnt["quartets"] == npair * (npair + 1) // 2
    assert np.abs(K - K.T).max() == 0.0
    assert np.trace(s.P @ K) > 0
    # Schwarz factors = sqrt of the largest diagonal over the shell pair
    bfo = s.bf_offsets()
    p = 0
    for I in range(s.nshell):
        for J in range(I + 1):
            ni, nj = 2 * s.shell_l[I] + 1, 2 * s.shell_l[J] + 1
            blk = D[bfo[I]:bfo[I] + ni, bfo[J]:bfo[J] + nj]
            assert abs(Q[p] - math.sqrt(blk.max())) <= 1e-15 * Q[p]
            p += 1


def test_sp8_cluster_K_brute_force_both_operators():
    s = hi.sp8_cluster()
    for omega in (0.0, hi.OMEGA_HSE):
        G = oracle.eri_tensor(s, omega=omega)
        Kb = np.einsum("ijkl,jl->ik", G, s.P)
        K, _, cnt = oracle.build_K(s, tau=0.0, omega=omega)
        assert np.abs(K - Kb).max() < 1e-13
        assert cnt["quartets"] == 136 * 137 // 2
        assert np.trace(s.P @ K) > 0


# ------------------------------------------------ Coulomb J (next row) ----
@pytest.mark.parametrize("omega", [0.0, 0.11])
def test_J_brute_force_and_coulomb_energy(small_spd, omega):
    """J from the unique quartets equals the n^4 contraction
    J_ij = sum_kl (ij|kl) P_kl; J is symmetric; the Coulomb energy
    sum_ijkl P_ij (ij|kl) P_kl is non-negative for any symmetric P (the kernel
    1/r and erfc(omega r)/r is positive definite); K from the joint build is
    the exchange of the K-only build."""
    s = small_spd
    G = oracle.eri_tensor(s, omega=omega)
    J, K, Q, cnt = oracle.build_JK(s, tau=0.0, omega=omega)
    Jb = np.einsum("ijkl,kl->ij", G, s.P)
    assert np.abs(J - Jb).max() <= 1e-13 * np.abs(Jb).max()
    assert np.abs(J - J.T).max() == 0.0
    K1, _, cnt1 = oracle.build_K(s, tau=0.0, omega=omega)
    assert np.abs(K - K1).max() <= 1e-14 * np.abs(K1).max()
    assert cnt["quartets"] == cnt1["quartets"] and (cnt["per_class"] == cnt1["per_class"]).all()
    rng = np.random.default_rng(5)
    for _ in range(3):
        A = rng.standard_normal((s.nbf, s.nbf))
        Ps = A + A.T
        Jr, _, _, _ = oracle.build_JK(s, tau=0.0, omega=omega, P=Ps)
        assert np.sum(Ps * Jr) >= -1e-12 * np.abs(Jr).max()


def test_J_single_s_function_closed_form():
    """One normalised s function with P = [[p]]: J = K = p (ss|ss), the
    one-centre value of the golden table."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "one_centre_ssss.txt")) if l.strip() and not l.startswith("#")]
    s = _one_shell_sys([[0, 0, 0]], [0], [[1.0]])
    s.P = np.array([[0.7]])
    for om, val in rows:
        J, K, _, _ = oracle.build_JK(s, tau=0.0, omega=float(om))
        assert abs(J[0, 0] - 0.7 * float(val)) < 1e-15
        assert abs(K[0, 0] - 0.7 * float(val)) < 1e-15


def test_J_sp8_cluster_brute_force():
    s = hi.sp8_cluster()
    G = oracle.eri_tensor(s, omega=hi.OMEGA_HSE)
    J, _, _, cnt = oracle.build_JK(s, tau=0.0, omega=hi.OMEGA_HSE)
    assert np.abs(J - np.einsum("ijkl,kl->ij", G, s.P)).max() < 1e-13
    assert cnt["quartets"] == 136 * 137 // 2


def test_screening_error_bound():
    """K(tau) - K(0) is bounded by the dropped quartets' Schwarz bounds."""
    s = hi.sp8_cluster()
    K0, Q, _ = oracle.build_K(s, tau=0.0, omega=0.11)
    for tau in (1e-6, 1e-4, 1e-2):
        Kt, _, cnt = oracle.build_K(s, tau=tau, omega=0.11)
        npair = len(Q)
        qq = np.outer(Q, Q)
        dropped = np.tril(qq < tau)
        nmax = 9  # at most 3x3 functions in a (pp) pair
        bound = 2 * 4 * nmax * np.abs(s.P).max() * qq[dropped].sum()
        assert np.abs(Kt - K0).max() <= bound + 1e-15
        assert cnt["quartets"] == int(np.tril(qq >= tau).sum())


def test_omega_limits(small_spd):
    s = small_spd
    a = oracle.shell_quartet(s, 2, 1, 5, 4, omega=0.0)
    b = oracle.shell_quartet(s, 2, 1, 5, 4, omega=1e-300)
    assert np.array_equal(a, b) or np.abs(a - b).max() < 1e-300
    c = oracle.shell_quartet(s, 2, 1, 5, 4, omega=1e5)
    assert np.abs(c).max() < 1e-5 * np.abs(a).max()
    d = oracle.shell_quartet(s, 2, 1, 5, 4, omega=0.11)
    # the attenuated kernel is pointwise smaller than 1/r: diagonal integrals drop
    dd = oracle.shell_quartet(s, 2, 2, 2, 2, omega=0.11)
    d0 = oracle.shell_quartet(s, 2, 2, 2, 2, omega=0.0)
    assert (np.einsum("ijij->ij", dd) < np.einsum("ijij->ij", d0)).all()
    assert d.shape == a.shape


def test_translation_rotation_homogeneity(small_spd):
    s = small_spd
    ref = oracle.eri_tensor(s, omega=0.11)
    t = hi._pack(s.xyz + np.array([3.1, -2.0, 0.7]),
                 [(int(s.shell_atom[i]), int(s.shell_l[i]),
                   s.exps[s.shell_off[i]:s.shell_off[i] + s.shell_nprim[i]],
                   s.coefs[s.shell_off[i]:s.shell_off[i] + s.shell_nprim[i]]) for i in range(s.nshell)],
                 s.P, {})
    assert np.abs(oracle.eri_tensor(t, omega=0.11) - ref).max() < 1e-13
    # homogeneity: exponents * lam^2, coordinates / lam, omega * lam -> integrals * lam
    lam = 1.7
    h = hi._pack(s.xyz / lam,
                 [(int(s.shell_atom[i]), int(s.shell_l[i]),
                   s.exps[s.shell_off[i]:s.shell_off[i] + s.shell_nprim[i]] * lam ** 2,
                   s.coefs[s.shell_off[i]:s.shell_off[i] + s.shell_nprim[i]]) for i in range(s.nshell)],
                 s.P, {})
    assert np.abs(oracle.eri_tensor(h, omega=0.11 * lam) - lam * ref).max() < 1e-12 * np.abs(ref).max()
    # rotation about z by 90 deg: p block (x,y,z) -> (y,-x,z) acts on p indices
    R = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    r = hi._pack(s.xyz @ R.T,
                 [(int(s.shell_atom[i]), int(s.shell_l[i]),
                   s.exps[s.shell_off[i]:s.shell_off[i] + s.shell_nprim[i]],
                   s.coefs[s.shell_off[i]:s.shell_off[i] + s.shell_nprim[i]]) for i in range(s.nshell)],
                 s.P, {})
    G2 = oracle.eri_tensor(r, omega=0.11)
    # s-s-s-s sub-blocks unchanged; full tensor has the same Frobenius norm
    sidx = s.bf_offsets()[s.shell_l == 0]
    assert np.abs(G2[np.ix_(sidx, sidx, sidx, sidx)] - ref[np.ix_(sidx, sidx, sidx, sidx)]).max() < 1e-13
    assert abs(np.linalg.norm(G2) - np.linalg.norm(ref)) < 1e-12 * np.linalg.norm(ref)
    # p functions rotate like vectors: (p s|s s) components of atom 0's p shell
    pidx = s.bf_offsets()[1] + np.arange(3)
    s0 = sidx[1]
    v = ref[pidx, s0, s0, s0]
    v2 = G2[pidx, s0, s0, s0]
    assert np.abs(v2 - R @ v).max() < 1e-13


def test_si64_basis_counts():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "si64_basis_counts.txt")) if l.strip() and not l.startswith("#")]
    for basis, nsh, nbf in rows:
        s = hi.si64_like(basis)
        assert s.nshell == int(nsh) and s.nbf == int(nbf)


def test_config_sizes():
    c0 = hi.sp8_cluster()
    assert c0.nshell == 16 and c0.nbf == 32
    c1 = hi.dzp256_lattice()
    assert c1.nshell == 1280 and c1.nbf == 3328 and c1.natom == 256
    assert np.allclose(c1.P, c1.P.T)


# ------------------------------ McMurchie-Davidson evaluation (all classes) ----
# A second, independent route to the same integrals (Hermite expansion of the
# Gaussian products, Hermite Coulomb integrals R_tuv), written here from the
# textbook formulation and sharing nothing with the oracle's Obara-Saika /
# Head-Gordon-Pople code.  For the attenuated kernel the Hermite seeds are
# (-2 rho)^n G_n with G_n = F_n(T) - theta^(2n+1) F_n(theta^2 T): the R
# recursion is linear in its seeds and holds separately for the two Coulomb-
# like terms F_0(rho r^2) and theta F_0(theta^2 rho r^2).
def _md_hermite_E(la, lb, a, b, Ax, Bx):
    """E[i][j][t] of the 1-D product x_A^i x_B^j exp(-a x_A^2 - b x_B^2)."""
    p = a + b
    mu = a * b / p
    X = Ax - Bx
    XPA, XPB = -b / p * X, a / p * X
    E = np.zeros((la + 1, lb + 1, la + lb + 2))
    E[0, 0, 0] = math.exp(-mu * X * X)
    for i in range(la + 1):
        for j in range(lb + 1):
            if i == 0 and j == 0:
                continue
            for t in range(i + j + 1):
                if j == 0:
                    prev, x = E[i - 1, 0], XPA
                else:
                    prev, x = E[i, j - 1], XPB
                v = x * prev[t] + (t + 1) * prev[t + 1]
                if t > 0:
                    v += prev[t - 1] / (2 * p)
                E[i, j, t] = v
    return E


def _md_hermite_R(L, rho, PQ, omega):
    import functools

    mp.mp.dps = 30
    T = rho * float(np.dot(PQ, PQ))
    seeds = []
    th2 = omega * omega / (omega * omega + rho) if omega > 0 else 0.0
    for n in range(L + 1):
        g = _boys_mp(n, T)
        if omega > 0:
            g -= mp.mpf(th2) ** (n + mp.mpf(1) / 2) * _boys_mp(n, th2 * T)
        seeds.append(float((-2 * rho) ** n * g))

    @functools.lru_cache(maxsize=None)
    def r(n, t, u, v):
        if t < 0 or u < 0 or v < 0:
            return 0.0
        if t == 0 and u == 0 and v == 0:
            return seeds[n]
        if t > 0:
            return (t - 1) * r(n + 1, t - 2, u, v) + PQ[0] * r(n + 1, t - 1, u, v)
        if u > 0:
            return (u - 1) * r(n + 1, t, u - 2, v) + PQ[1] * r(n + 1, t, u - 1, v)
        return (v - 1) * r(n + 1, t, u, v - 2) + PQ[2] * r(n + 1, t, u, v - 1)

    return r


def _md_cart_monomials(l):
    return [(i, j, l - i - j) for i in range(l, -1, -1) for j in range(l - i, -1, -1)]


def _md_spherical_block(ls, cen, prims, omega):
    """Contracted spherical block [i][j][k][l] of four shells by
    McMurchie-Davidson; prims[s] = list of (exponent, coefficient) where the
    coefficient already contains the x^l primitive normalisation."""
    la, lb, lc, ld = ls
    L = sum(ls)
    cart = [_md_cart_monomials(l) for l in ls]
    ncart = [len(c) for c in cart]
    out_cart = np.zeros(ncart)
    for (a, ca) in prims[0]:
        for (b, cb) in prims[1]:
            p = a + b
            P = (a * cen[0] + b * cen[1]) / p
            Eb = [_md_hermite_E(la, lb, a, b, cen[0][x], cen[1][x]) for x in range(3)]
            for (c, cc) in prims[2]:
                for (d, cd) in prims[3]:
                    q = c + d
                    Q = (c * cen[2] + d * cen[3]) / q
                    Ek = [_md_hermite_E(lc, ld, c, d, cen[2][x], cen[3][x]) for x in range(3)]
                    rho = p * q / (p + q)
                    r = _md_hermite_R(L, rho, P - Q, omega)
                    pref = 2 * math.pi ** 2.5 / (p * q * math.sqrt(p + q)) * ca * cb * cc * cd
                    for ia, ma in enumerate(cart[0]):
                        for ib, mb in enumerate(cart[1]):
                            bra = {}
                            for t in range(ma[0] + mb[0] + 1):
                                for u in range(ma[1] + mb[1] + 1):
                                    for v in range(ma[2] + mb[2] + 1):
                                        bra[(t, u, v)] = (Eb[0][ma[0], mb[0], t] * Eb[1][ma[1], mb[1], u]
                                                          * Eb[2][ma[2], mb[2], v])
                            for ic, mc in enumerate(cart[2]):
                                for id_, md_ in enumerate(cart[3]):
                                    tot = 0.0
                                    for x in range(mc[0] + md_[0] + 1):
                                        for y in range(mc[1] + md_[1] + 1):
                                            for z in range(mc[2] + md_[2] + 1):
                                                e = (Ek[0][mc[0], md_[0], x] * Ek[1][mc[1], md_[1], y]
                                                     * Ek[2][mc[2], md_[2], z]) * (-1) ** (x + y + z)
                                                for (t, u, v), eb in bra.items():
                                                    tot += eb * e * r(0, t + x, u + y, v + z)
                                    out_cart[ia, ib, ic, id_] += pref * tot
    # spherical transform of every index (rows relative to x^l-normalised
    # Cartesians)
    mats = []
    for l, cl in zip(ls, cart):
        M = np.zeros((2 * l + 1, len(cl)))
        for m, row in enumerate(_SPH[l]):
            for mono, w in row:
                M[m, cl.index(mono)] = w
        mats.append(M)
    return np.einsum("ai,bj,ck,dl,ijkl->abcd", *mats, out_cart)


@pytest.mark.parametrize("ls", [(2, 2, 2, 1), (2, 2, 2, 2), (1, 2, 2, 2), (2, 1, 2, 1), (2, 2, 1, 1),
                                (2, 2, 2, 0), (2, 2, 0, 0), (1, 1, 1, 1), (2, 0, 1, 0), (0, 0, 0, 0)])
@pytest.mark.parametrize("omega", [0.0, 0.11])
def test_every_component_against_mcmurchie_davidson(ls, omega):
    """Every spherical component of single-primitive shell quartets, among
    them the two highest classes (dd|dp) (L = 7) and (dd|dd) (L = 8), equals a
    McMurchie-Davidson evaluation (Hermite expansion), a different textbook
    route to the integrals than the oracle's Obara-Saika recurrences, to 1e-12
    of the block's largest value."""
    rng = np.random.default_rng(sum(ls) * 31 + ls[0] * 7 + ls[3] + int(omega * 100))
    cen = rng.uniform(-1.5, 1.5, size=(4, 3))
    ex = rng.uniform(0.3, 2.0, size=4)
    s = _one_shell_sys(cen, list(ls), [[e] for e in ex])
    got = oracle.shell_quartet(s, 0, 1, 2, 3, omega=omega)
    prims = [[(ex[i], _norm_prim(ex[i], ls[i]))] for i in range(4)]
    ref = _md_spherical_block(ls, cen, prims, omega)
    scale = np.abs(ref).max()
    assert scale > 0
    assert np.abs(got - ref).max() <= 1e-12 * scale, (np.abs(got - ref).max(), scale)


@pytest.mark.parametrize("omega", [0.0, 0.11])
def test_contracted_high_class_against_mcmurchie_davidson(omega):
    """Contracted (dd|dp) with 2 primitives per shell: the primitive loop,
    contraction and horizontal recurrence of the oracle against the Hermite
    route summed over primitives."""
    ls = (2, 2, 2, 1)
    rng = np.random.default_rng(77 + int(omega * 100))
    cen = rng.uniform(-1.2, 1.2, size=(4, 3))
    exps = [rng.uniform(0.2, 3.0, size=2) for _ in range(4)]
    coefs = [rng.uniform(0.1, 1.0, size=2) for _ in range(4)]
    s = _one_shell_sys(cen, list(ls), exps, coefs)
    cn = oracle.normalised_coefs(s)
    got = oracle.shell_quartet(s, 0, 1, 2, 3, omega=omega)
    prims = [[(exps[i][k], cn[2 * i + k]) for k in range(2)] for i in range(4)]
    ref = _md_spherical_block(ls, cen, prims, omega)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_digest_list_reproduces_build_K():
    """The list digestion behind the CPU baseline: the screened unique quartets
    of sp8_cluster (p >= q, Q_p Q_q >= tau, by the oracle's own Schwarz factors)
    digested as a list, then K' + K'^T, equal the screened build_K (itself held
    to the brute-force n^4 contraction)."""
    s = hi.sp8_cluster()
    tau = 1e-10
    K, Q, cnt = oracle.build_K(s, tau=tau, omega=0.11)
    qmax = Q.max()
    keep = Q * qmax >= tau
    pq = [(p, q) for p in range(len(Q)) if keep[p] for q in range(p + 1) if keep[q] and Q[p] * Q[q] >= tau]
    assert len(pq) == cnt["quartets"]
    rng = np.random.default_rng(3)
    pq = np.asarray(pq, dtype=np.int64)[rng.permutation(len(pq))]
    Kp = oracle.digest_list(s, pq, omega=0.11)
    assert np.abs(Kp + Kp.T - K).max() <= 1e-14 * np.abs(K).max()


# ---------------------------------- density-weighted screening (next row) ----
def _shell_pmax_np(s, P):
    bfo = list(s.bf_offsets()) + [s.nbf]
    n = s.nshell
    M = np.zeros((n, n))
    for X in range(n):
        for Y in range(n):
            M[X, Y] = np.abs(P[bfo[X]:bfo[X + 1], bfo[Y]:bfo[Y + 1]]).max()
    return M


def _density_count(s, Q, P, tau, coulomb=False):
    """Unique quartets computed under the density-weighted rule, counted
    directly from the Schwarz factors and the shell-block maxima of |P|."""
    M = _shell_pmax_np(s, P)
    n = s.nshell
    pid = [(I, J) for I in range(n) for J in range(I + 1)]
    qmax = Q.max()
    keep = [p for p in range(len(pid)) if Q[p] * qmax >= tau]
    cnt = 0
    for a, p in enumerate(keep):
        I, J = pid[p]
        for q in keep[:a + 1]:
            if not (Q[p] * Q[q] >= tau):
                continue
            K, L = pid[q]
            d = max(M[I, K], M[I, L], M[J, K], M[J, L])
            if coulomb:
                d = max(d, M[I, J], M[K, L])
            if Q[p] * Q[q] * d >= tau:
                cnt += 1
    return cnt


@pytest.mark.parametrize("coulomb", [False, True])
def test_density_screening_counts_and_error_bound(coulomb):
    """The density-weighted build computes exactly the quartets the rule
    keeps (counted independently), and differs from the Schwarz-only build by
    at most what the dropped quartets can contribute: each value is bounded by
    Q_IJ Q_KL and meets |P| <= D in the digestion (<= 25 functions per shell
    pair, four images and the transpose)."""
    s = hi.lattice_system(6, seed=23, nprim_range=(1, 3))
    tau = 1e-7
    if coulomb:
        J0, K0, Q, c0 = oracle.build_JK(s, tau=tau, omega=0.11)
        Jd, Kd, Qd, cd = oracle.build_K_density(s, tau=tau, omega=0.11, coulomb=True)
    else:
        K0, Q, c0 = oracle.build_K(s, tau=tau, omega=0.11)
        Kd, Qd, cd = oracle.build_K_density(s, tau=tau, omega=0.11)
    assert np.array_equal(Q, Qd)
    want = _density_count(s, Q, s.P, tau, coulomb)
    assert cd["quartets"] == want
    assert 0 < cd["quartets"] < c0["quartets"]
    # dropped quartets: Schwarz-kept minus density-kept
    M = _shell_pmax_np(s, s.P)
    n = s.nshell
    pid = [(I, J) for I in range(n) for J in range(I + 1)]
    qmax = Q.max()
    bound = 0.0
    for p in range(len(pid)):
        if not Q[p] * qmax >= tau:
            continue
        I, J = pid[p]
        for q in range(p + 1):
            if not (Q[q] * qmax >= tau and Q[p] * Q[q] >= tau):
                continue
            K, L = pid[q]
            d = max(M[I, K], M[I, L], M[J, K], M[J, L])
            if coulomb:
                d = max(d, M[I, J], M[K, L])
            if not Q[p] * Q[q] * d >= tau:
                bound += 2 * 4 * 25 * Q[p] * Q[q] * d
    assert np.abs(Kd - K0).max() <= bound
    assert np.abs(Kd - Kd.T).max() == 0.0
    if coulomb:
        assert np.abs(Jd - J0).max() <= bound


def test_density_screening_reduces_to_schwarz_for_unit_blocks():
    """With every shell block of |P| peaking at exactly 1 the density weight
    is 1 and the rule is the Schwarz rule: same quartets, same K."""
    s = hi.lattice_system(5, seed=24, nprim_range=(1, 3))
    P = np.ones((s.nbf, s.nbf))
    K0, Q, c0 = oracle.build_K(s, tau=1e-8, omega=0.11, P=P)
    Kd, _, cd = oracle.build_K_density(s, tau=1e-8, omega=0.11, P=P)
    assert cd["quartets"] == c0["quartets"]
    assert (cd["per_class"] == c0["per_class"]).all()
    assert np.abs(Kd - K0).max() <= 1e-14 * np.abs(K0).max()


def test_density_screening_tau_zero_keeps_everything():
    s = hi.sp8_cluster()
    K0, Q, c0 = oracle.build_K(s, tau=0.0, omega=0.11)
    Kd, _, cd = oracle.build_K_density(s, tau=0.0, omega=0.11)
    assert cd["quartets"] == c0["quartets"] == 136 * 137 // 2
    assert np.abs(Kd - K0).max() <= 1e-14 * np.abs(K0).max()


# ------------------------------------------- periodic exchange (next row) ----
def test_periodic_home_cell_only_is_the_molecular_build():
    """A cluster of the home cell alone: the periodic sum is the molecular
    exchange matrix (every row, every column)."""
    cl = hi.periodic_cluster(natom_cell=3, reach=(0, 0, 0), lmax=2, nprim_range=(1, 3))
    assert cl.meta["nhome_shell"] == cl.nshell
    Kp, cnt = oracle.build_K_periodic(cl, tau=1e-10, omega=0.11)
    Km, Q, cm = oracle.build_K(cl, tau=1e-10, omega=0.11)
    assert Kp.shape == Km.shape
    assert np.abs(Kp - Km).max() <= 1e-13 * np.abs(Km).max()
    # combinations of two (unordered) pairs in either order: twice the unique
    # quartets less the diagonal ones
    assert cnt["quartets"] == 2 * cm["quartets"] - int((Q * Q >= 1e-10).sum())


def test_periodic_equals_brute_force_tensor_and_cluster_rows():
    """tau = 0 over a three-cell chain: K^G_{mu lambda} = sum_{j,l} (mu j|lambda l)
    Pbig[j][l] from the n^4 ERI tensor of the whole cluster, and the home-cell
    rows of the molecular build of the cluster (itself pinned to the tensor)."""
    cl = hi.periodic_cluster(natom_cell=1, reach=(1, 0, 0), lmax=1, nprim_range=(1, 2))
    nh = int(np.sum(2 * cl.shell_l[:cl.meta["nhome_shell"]] + 1))
    Kp, cnt = oracle.build_K_periodic(cl, tau=0.0, omega=0.11)
    G = oracle.eri_tensor(cl, omega=0.11)
    Kb = np.einsum("ijkl,jl->ik", G[:nh], cl.P)
    assert np.abs(Kp - Kb).max() <= 1e-13 * np.abs(Kb).max()
    Km, _, _ = oracle.build_K(cl, tau=0.0, omega=0.11)
    assert np.abs(Kp - Km[:nh]).max() <= 1e-13 * np.abs(Km).max()
    npair = cl.nshell * (cl.nshell + 1) // 2
    nhs = cl.meta["nhome_shell"]
    home_pairs = sum(1 for I in range(cl.nshell) for J in range(I + 1) if I < nhs or J < nhs)
    assert cnt["quartets"] == home_pairs * npair


def test_periodic_counts_and_screening_bound():
    """27 cells: the screened combinations equal a direct count from the
    Schwarz factors, and the screened K differs from the tau = 0 K by at most
    what the dropped quartets can contribute."""
    cl = hi.periodic_cluster(natom_cell=1, reach=(1, 1, 1), lmax=1, nprim_range=(1, 2))
    tau = 1e-6
    Kp, cnt = oracle.build_K_periodic(cl, tau=tau, omega=0.11)
    K0, _ = oracle.build_K_periodic(cl, tau=0.0, omega=0.11)
    Q = oracle.schwarz(cl, omega=0.11)
    nhs = cl.meta["nhome_shell"]
    pid = [(I, J) for I in range(cl.nshell) for J in range(I + 1)]
    home = np.array([I < nhs or J < nhs for (I, J) in pid])
    qq = np.outer(Q[home], Q)
    assert cnt["quartets"] == int((qq >= tau).sum())
    # each dropped (ordered) shell quartet adds at most Q_IJ Q_KL max|P| per
    # function pair, <= 3 x 3 functions for s/p shells, both ket orders
    bound = 2 * 9 * np.abs(cl.P).max() * qq[qq < tau].sum() * 2
    assert 0 < np.abs(Kp - K0).max() <= bound
