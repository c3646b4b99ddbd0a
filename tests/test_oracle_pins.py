"""Pins of the FP64 oracle to facts the paper and the mathematics fix.

None of these checks re-types the oracle's formula: each compares it against
an independent route (a library FFT, a closed form, an identity between two
different oracle entry points, a plain Python loop, finite differences, or the
Madelung constant the paper prints).  Together they catch a dropped term, a
wrong sign, a wrong index centring or a transposed operand.
"""
import cmath
import math
import os

import numpy as np
import pytest

import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _kgrid(N):
    axes = [np.arange(n) - n // 2 for n in N]
    return np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1)


@pytest.mark.parametrize("N", [(8,), (6, 4), (4, 6, 8), (2, 2, 2)])
def test_equispaced_points_equal_dft(oracle_mod, N):
    """Eq. (5) on x_j = j/N, j in I_N (M = #I_N) is the DFT of Eq. (3);
    checked against numpy's FFT with centred index maps (Section 1)."""
    g = W.rng(11)
    N = tuple(N)
    j = _kgrid(N).reshape(-1, len(N))
    x = j / np.asarray(N, dtype=np.float64)
    F = W.complex_normal(j.shape[0], g).reshape(N)
    got = oracle_mod.ndft_adjoint(N, x, F.reshape(-1))
    ref = np.fft.fftshift(np.fft.fftn(np.fft.ifftshift(F)))
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))
    # Eq. (4): the inverse DFT is 1/#I_N times Eq. (6) on the same points.
    back = oracle_mod.ndft_forward(N, x, ref) / np.prod(N)
    assert np.max(np.abs(back - F.reshape(-1))) <= 1e-13 * np.max(np.abs(F))


def test_single_point_is_pure_exponential(oracle_mod):
    """M = 1, f = 1: Eq. (5) reduces to exp(-2 pi i k.x0)."""
    g = W.rng(12)
    N = (6, 8, 4)
    x0 = W.uniform_points(1, 3, g)
    got = oracle_mod.ndft_adjoint(N, x0, np.ones(1))
    k = _kgrid(N)
    ref = np.exp(-2j * np.pi * (k @ x0[0]))
    assert np.max(np.abs(got - ref)) <= 1e-14
    # Eq. (6) at one point with fhat = delta_k gives exp(+2 pi i k.x0).
    fh = np.zeros(N, dtype=np.complex128)
    fh[4, 1, 3] = 1.0
    kk = np.array([4 - 3, 1 - 4, 3 - 2])
    got1 = oracle_mod.ndft_forward(N, x0, fh)
    assert abs(got1[0] - np.exp(2j * np.pi * (kk @ x0[0]))) <= 1e-14


def test_points_at_origin_sum_values(oracle_mod):
    """All points at x = 0: every frequency equals sum_j f_j."""
    g = W.rng(13)
    f = W.complex_normal(7, g)
    got = oracle_mod.ndft_adjoint((4, 4, 4), np.zeros((7, 3)), f)
    assert np.max(np.abs(got - f.sum())) <= 1e-14 * np.abs(f).sum()


def test_adjoint_identity(oracle_mod):
    """<A f, g> = <f, A^H g> for the matrix of Eq. (5) and its transpose
    Eq. (6) (Section 1, the matrix form)."""
    g = W.rng(14)
    N = (8, 6, 10)
    x = W.uniform_points(300, 3, g)
    f = W.complex_normal(300, g)
    h = W.complex_normal(int(np.prod(N)), g).reshape(N)
    Af = oracle_mod.ndft_adjoint(N, x, f)
    AHh = oracle_mod.ndft_forward(N, x, h)
    lhs = np.vdot(h.reshape(-1), Af.reshape(-1))
    rhs = np.vdot(AHh, f)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def _brute_adjoint(N, x, f):
    out = {}
    for k0 in range(-N[0] // 2, N[0] // 2):
        for k1 in range(-N[1] // 2, N[1] // 2):
            for k2 in range(-N[2] // 2, N[2] // 2):
                s = 0j
                for j in range(len(f)):
                    s += f[j] * cmath.exp(-2j * math.pi * (k0 * x[j][0] + k1 * x[j][1] + k2 * x[j][2]))
                out[(k0, k1, k2)] = s
    return out


def test_brute_force_tiny(oracle_mod):
    """M <= 8, N <= 4^3: the oracle against a scalar Python triple loop."""
    g = W.rng(15)
    N = (4, 2, 4)
    x = W.uniform_points(8, 3, g)
    f = W.complex_normal(8, g)
    got = oracle_mod.ndft_adjoint(N, x, f)
    ref = _brute_adjoint(N, x.tolist(), f.tolist())
    for (k0, k1, k2), v in ref.items():
        assert abs(got[k0 + N[0] // 2, k1 + N[1] // 2, k2 + N[2] // 2] - v) <= 1e-13
    # Eq. (6) brute force on the same tiny case.
    fh = W.complex_normal(int(np.prod(N)), g).reshape(N)
    gotf = oracle_mod.ndft_forward(N, x, fh)
    for j in range(8):
        s = 0j
        for (k0, k1, k2) in ref:
            s += fh[k0 + 2, k1 + 1, k2 + 2] * cmath.exp(2j * math.pi * (k0 * x[j][0] + k1 * x[j][1] + k2 * x[j][2]))
        assert abs(gotf[j] - s) <= 1e-13


def test_sampled_outputs_match_full(oracle_mod):
    g = W.rng(16)
    N = (6, 6, 8)
    x = W.uniform_points(50, 3, g)
    f = W.complex_normal(50, g)
    full = oracle_mod.ndft_adjoint(N, x, f).reshape(-1)
    idx = W.sample_indices(full.size, 17, g)
    assert np.array_equal(oracle_mod.ndft_adjoint(N, x, f, kidx=idx), full[idx])
    fh = W.complex_normal(full.size, g)
    fullf = oracle_mod.ndft_forward(N, x, fh)
    jdx = W.sample_indices(50, 9, g)
    assert np.array_equal(oracle_mod.ndft_forward(N, x, fh, jidx=jdx), fullf[jdx])


def test_shift_theorem(oracle_mod):
    """x -> x + s (wrapped) multiplies fhat(k) by exp(-2 pi i k.s)."""
    g = W.rng(17)
    N = (8, 4, 6)
    x = W.uniform_points(40, 3, g)
    f = W.complex_normal(40, g)
    s = np.array([0.125, -0.3, 0.41])
    a = oracle_mod.ndft_adjoint(N, x, f)
    b = oracle_mod.ndft_adjoint(N, W.wrap_unit(x + s), f)
    ph = np.exp(-2j * np.pi * (_kgrid(N) @ s))
    assert np.max(np.abs(b - a * ph)) <= 1e-12 * np.max(np.abs(a))


def test_subcell_decomposition_eq8(oracle_mod):
    """Eq. (8): the transform of all points equals the sum of the transforms
    of the points of each subcell (here: 4 slabs along the first axis)."""
    g = W.rng(18)
    N = (8, 8, 8)
    x = W.uniform_points(400, 3, g)
    f = W.complex_normal(400, g)
    whole = oracle_mod.ndft_adjoint(N, x, f)
    cell = np.floor((x[:, 0] + 0.5) * 4).astype(int)
    parts = sum(oracle_mod.ndft_adjoint(N, x[cell == i], f[cell == i]) for i in range(4))
    assert np.max(np.abs(parts - whole)) <= 1e-12 * np.max(np.abs(whole))


def test_gradient_matches_finite_differences(oracle_mod):
    """Analytic gradient of L = sum_k c_k |fhat_k|^2 + Re<w, fhat> through
    Eq. (5), against central finite differences of the oracle itself."""
    g = W.rng(19)
    N = (6, 4, 8)
    M = 12
    x = W.uniform_points(M, 3, g) * 0.9
    f = W.complex_normal(M, g)
    c = g.random(N)
    w = W.complex_normal(int(np.prod(N)), g).reshape(N)

    def loss(xx, ff):
        fh = oracle_mod.ndft_adjoint(N, xx, ff)
        return float(np.sum(c * np.abs(fh) ** 2) + np.real(np.vdot(w, fh)))

    fh = oracle_mod.ndft_adjoint(N, x, f)
    gbar = 2 * c * fh + w               # dL/dRe fhat + i dL/dIm fhat
    gf, gx = oracle_mod.ndft_adjoint_grad(N, x, f, gbar)
    h = 1e-6
    for j in (0, 5, 11):
        for t in range(3):
            xp = x.copy(); xp[j, t] += h
            xm = x.copy(); xm[j, t] -= h
            fd = (loss(xp, f) - loss(xm, f)) / (2 * h)
            assert abs(fd - gx[j, t]) <= 1e-6 * max(1.0, abs(fd))
        fp = f.copy(); fp[j] += h
        fm = f.copy(); fm[j] -= h
        dre = (loss(x, fp) - loss(x, fm)) / (2 * h)
        fp = f.copy(); fp[j] += 1j * h
        fm = f.copy(); fm[j] -= 1j * h
        dim = (loss(x, fp) - loss(x, fm)) / (2 * h)
        assert abs((dre + 1j * dim) - gf[j]) <= 1e-6 * max(1.0, abs(gf[j]))


def test_rel_l2_metric(oracle_mod):
    """Eq. (9) on a case with a known answer."""
    s = np.array([3 + 4j, 0j])
    a = np.array([3 + 4j, 1j])
    assert abs(oracle_mod.rel_l2(a, s) - 0.2) <= 1e-15


def _gold():
    vals = {}
    with open(os.path.join(GOLD, "madelung_fluorite.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                k, v = line.split()
                vals[k] = float(v)
    return vals


def test_fluorite_madelung_matches_paper(oracle_mod):
    """Direct Ewald (Eqs. (11)-(12)) on a 2x2x2 fluorite supercell gives the
    Madelung constant the paper prints, for every alpha in its range, and the
    total is alpha-independent (Section 5)."""
    gold = _gold()
    r, q, L = W.fluorite(2)
    vals = []
    for alpha in (gold["alpha_min"], 1.5, gold["alpha_max"]):
        kmax = int(math.ceil(6.2 * alpha * L / math.pi))
        U = oracle_mod.ewald_real(r, q, L, alpha, 3) + oracle_mod.ewald_recip(r, q, L, alpha, kmax)
        vals.append(oracle_mod.madelung_from_energy(U, q.size))
    for v in vals:
        assert abs(v - gold["madelung"]) <= 5e-5
    assert max(vals) - min(vals) <= 1e-9


def test_ewald_forces_match_finite_differences(oracle_mod):
    """Forces of Eqs. (11)-(12) against central differences of the energy."""
    r, q, L = W.fluorite(1, displacement_std=0.05, seed=21)
    alpha = 1.6
    kmax = int(math.ceil(6.2 * alpha * L / math.pi))

    def energy(rr):
        return oracle_mod.ewald_real(rr, q, L, alpha, 4) + oracle_mod.ewald_recip(rr, q, L, alpha, kmax)

    _, Fr = oracle_mod.ewald_real(r, q, L, alpha, 4, forces=True)
    Fk = oracle_mod.ewald_recip_forces(r, q, L, alpha, kmax)
    F = Fr + Fk
    h = 1e-5
    for i in (0, 3, 7):
        for t in range(3):
            rp = r.copy(); rp[i, t] += h
            rm = r.copy(); rm[i, t] -= h
            fd = -(energy(rp) - energy(rm)) / (2 * h)
            assert abs(fd - F[i, t]) <= 1e-6 * max(1.0, abs(fd))
    # Newton's third law: the net force vanishes.
    assert np.max(np.abs(F.sum(axis=0))) <= 1e-9


def test_selected_ion_ewald_forces(oracle_mod):
    """The selected-ions variant of Eq. (12) gives the same energy as the full
    reciprocal sum and, for the listed ions, forces equal to central
    differences of that (Madelung-pinned) energy."""
    r, q, L = W.fluorite(1, displacement_std=0.05, seed=23)
    alpha = 1.6
    kmax = int(math.ceil(6.2 * alpha * L / math.pi))
    sel = np.array([5, 0, 9], dtype=np.int64)
    U, F, _ = oracle_mod.ewald_recip_selected(r, q, L, alpha, kmax, sel)
    assert abs(U - oracle_mod.ewald_recip(r, q, L, alpha, kmax)) <= 1e-12 * abs(U)
    h = 1e-5
    for a, i in enumerate(sel):
        for t in range(3):
            rp = r.copy(); rp[i, t] += h
            rm = r.copy(); rm[i, t] -= h
            fd = -(oracle_mod.ewald_recip(rp, q, L, alpha, kmax) - oracle_mod.ewald_recip(rm, q, L, alpha, kmax)) / (2 * h)
            assert abs(fd - F[a, t]) <= 1e-6 * max(1.0, abs(fd))
