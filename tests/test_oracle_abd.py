"""Pins of the oracle's Sec. 6 path: cell ("consistent") damping
Im H = omega sum_cells r_cell M_cell, the frequency adapted backward-differences
damped leapfrog I_abd (Def. 6) and S_T^abd (Def. 7)."""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle
from paper_2006_16861_amd import inputs


def sine_mode(n, p):
    axes = [np.sin(math.pi * pa * (np.arange(na) + 1) / (na + 1)) for na, pa in zip(n, p)]
    e = axes[0]
    for ax in axes[1:]:
        e = np.multiply.outer(e, ax)
    return e


def symbols(ndim, t):
    """Symbols of the assembled compact tables (S for h^2 Re-stiffness, M mass)."""
    c = [math.cos(x) for x in t]
    if ndim == 2:
        return (20 - 8 * c[0] - 8 * c[1] - 4 * c[0] * c[1]) / 6, 2 / 3 + (c[0] + c[1]) / 6
    pair = c[0] * c[1] + c[0] * c[2] + c[1] * c[2]
    return (24 - 4 * sum(c) - 4 * pair) / 6, 0.5 + sum(c) / 6


def cell_mean(a):
    """Mean over each cell's corners, indices clamped into the box (all n+1 cells)."""
    d = a.ndim
    pad = np.pad(a, 1, mode="edge")
    out = np.zeros(tuple(s + 1 for s in a.shape))
    for corner in np.ndindex(*(2,) * d):
        out += pad[tuple(slice(o, o + s + 1) for o, s in zip(corner, a.shape))]
    return out / 2 ** d


def problem(n, seed, rscale=2.0):
    p = inputs.random_medium(n, seed=seed, width=2, r_scale=rscale)
    rng = np.random.default_rng(seed + 7)
    R = p.R + rng.uniform(0.0, 0.3 * p.omega, p.n)      # damping everywhere, non-uniform
    return p, R


@pytest.mark.parametrize("n", [(9, 11), (5, 4, 6)])
def test_cell_damping_matches_element_assembly(n):
    p, R = problem(n, 50)
    o = oracle.Op(p.n, p.h, p.omega, p.c, R, damping="cell")
    H = oracle.assemble_H(p.n, p.h, p.omega, p.c, R, damping="cell")
    rng = np.random.default_rng(1)
    x = rng.standard_normal(p.n) + 1j * rng.standard_normal(p.n)
    y = (H @ x.reshape(-1)).reshape(p.n)
    assert np.linalg.norm(o.apply_H(x) - y) <= 1e-12 * np.linalg.norm(y)
    Hi = H.imag.toarray()
    assert np.allclose(Hi, Hi.T, rtol=0, atol=1e-12 * abs(Hi).max())
    assert abs((H.imag - H.imag.multiply(np.eye(H.shape[0]))).sum()) > 0    # not diagonal


@pytest.mark.parametrize("ndim", [2, 3])
def test_cell_damping_sine_modes(ndim):
    """Constant c and R: sine modes are eigenvectors of H with eigenvalue
    h^-2 S(t) - k^2 M(t) + i omega R M(t)."""
    n = (7, 9) if ndim == 2 else (5, 4, 6)
    h, omega, cval, Rval = 1.0 / 10, 17.0, 1.3, 2.5
    o = oracle.Op(n, h, omega, np.full(n, cval), np.full(n, Rval), damping="cell")
    k2 = (omega / cval) ** 2
    for p in [(1,) * ndim, tuple(range(2, 2 + ndim)), n]:
        e = sine_mode(n, p)
        t = [math.pi * pa / (na + 1) for na, pa in zip(n, p)]
        S, M = symbols(ndim, t)
        lam = S / h ** 2 - k2 * M + 1j * omega * Rval * M
        He = o.apply_H(e.astype(np.complex128))
        assert np.linalg.norm(He - lam * e) <= 1e-12 * abs(lam) * np.linalg.norm(e)


def dense(apply, n):
    N = int(np.prod(n))
    A = np.zeros((N, N))
    for j in range(N):
        x = np.zeros(N)
        x[j] = 1.0
        A[:, j] = apply(x.reshape(n)).reshape(-1)
    return A


def stable(theta, kmax2, lam_s, lam_im):
    alpha = theta ** 2 / (4 * math.sin(theta / 2) ** 2)
    beta = theta / math.sin(theta)
    w2 = kmax2 + beta / theta * (1 - math.cos(theta)) * lam_im
    lhs = theta ** 2 / alpha * (lam_s / w2 + 1) + theta * beta / alpha * (1 + math.cos(theta)) * lam_im / w2
    return lhs < 4, w2


@pytest.mark.parametrize("n", [(8, 7), (4, 5, 3)])
@pytest.mark.parametrize("rscale", [0.5, 2.0, 8.0])
def test_abd_parameters_and_stability_conditions(n, rscale):
    """Sec. 6.1: omega^2 = k_max^2 + (beta/theta)(1 - cos theta) lambda_max(Im H)
    makes K >= 0; n_P is the smallest multiple of 4 with 4I - K - 2L > 0 (from the
    bounds); L >= 0.  Checked with the dense K and L."""
    p, R = problem(n, 60, rscale)
    o = oracle.Op(p.n, p.h, p.omega, p.c, R, damping="cell")
    kmax2 = p.omega ** 2 * cell_mean(1.0 / p.c ** 2).max()
    lam_im = p.omega * cell_mean(R).max()
    lam_s = (16 / 3) / p.h ** 2        # max of the compact stiffness symbol (2-D and 3-D)
    ok, w2 = stable(2 * math.pi / o.nP, kmax2, lam_s, lam_im)
    assert ok
    if o.nP > 4:
        assert not stable(2 * math.pi / (o.nP - 4), kmax2, lam_s, lam_im)[0]
    assert abs(o.omega_c ** 2 - w2) <= 1e-12 * w2
    assert abs(o.omega_c * o.dt - 2 * math.pi / o.nP) <= 1e-14
    K = dense(o.apply_K, p.n)
    L = dense(o.apply_L, p.n)
    assert np.allclose(K, K.T, atol=1e-13 * abs(K).max())
    assert np.linalg.eigvalsh(K).min() >= -1e-12 * abs(K).max()
    assert np.linalg.eigvalsh(L).min() >= -1e-13 * max(abs(L).max(), 1e-300)
    assert np.linalg.eigvalsh(4 * np.eye(K.shape[0]) - K - 2 * L).min() > 0


@pytest.mark.parametrize("n", [(10, 12), (5, 6, 4)])
def test_abd_harmonic_invariance(n):
    """Prop. 5.1: with U = H^-1 F, u_n = Re(e^{i omega n dt} U) satisfies the
    I_abd recurrence forced by Re(e^{i omega n dt} F) at every step (omega the
    computational frequency)."""
    p, R = problem(n, 70)
    o = oracle.Op(p.n, p.h, p.omega, p.c, R, damping="cell")
    H = oracle.assemble_H(p.n, p.h, p.omega, p.c, R, damping="cell")
    rng = np.random.default_rng(3)
    F = rng.standard_normal(p.n) + 1j * rng.standard_normal(p.n)
    U = spla.spsolve(H.tocsc(), F.reshape(-1)).reshape(p.n)
    wdt = o.omega_c * o.dt
    u = lambda k: np.real(np.exp(1j * wdt * k) * U)
    f = lambda k: np.real(np.exp(1j * wdt * k) * F)
    for k in range(0, 12):
        up = o.step(u(k), u(k - 1), f(k))
        assert np.linalg.norm(up - u(k + 1)) <= 1e-11 * np.linalg.norm(u(k + 1))


@pytest.mark.parametrize("n", [(12, 9), (5, 4, 6)])
def test_abd_energy_identity_and_conservation(n):
    """Sec. 6.2: E_bd(n+1/2) - E_bd(n-1/2) = -2 <u+ - u-, L (u+ - u-)> (<= 0 for
    L >= 0), and E_bd is conserved without damping."""
    for rs in (2.0, 0.0):
        p, R = problem(n, 80)
        R = R * (rs > 0)
        o = oracle.Op(p.n, p.h, p.omega, p.c, R, damping="cell")
        rng = np.random.default_rng(4)
        um, u = rng.standard_normal(p.n), rng.standard_normal(p.n)

        def E(a, b):
            dlt, sig = a - b, a + b
            return (np.vdot(dlt, 4 * dlt - o.apply_K(dlt)) + np.vdot(sig, o.apply_K(sig))
                    - 2 * np.vdot(dlt, o.apply_L(dlt)))
        e0 = E(u, um)
        e = e0
        for _ in range(60):
            up = o.step(u, um, None)
            e1 = E(up, u)
            d = up - um
            assert abs((e1 - e) + 2 * np.vdot(d, o.apply_L(d))) <= 1e-11 * abs(e0)
            if rs == 0:
                assert abs(e1 - e0) <= 1e-11 * abs(e0)
            else:
                assert e1 <= e + 1e-12 * abs(e0)
            um, u, e = u, up, e1


@pytest.mark.parametrize("ndim", [2, 3])
def test_abd_precond_on_eigenvector_is_scalar_recurrence(ndim):
    """Constant c and R: for F = e_p, S_T^abd F = s e_p where s is the scalar
    I_abd recurrence of the mode (K_p, L_p from the eigenvalues of Re H and
    Im H) driven by chi(1 - j/N_s) e^{i 2 pi j/n_P}."""
    n = (9, 8) if ndim == 2 else (5, 6, 4)
    h, omega, cval, Rval = 1.0 / 10, 11.0, 1.1, 3.0
    o = oracle.Op(n, h, omega, np.full(n, cval), np.full(n, Rval), damping="cell")
    p = (2,) * ndim
    e = sine_mode(n, p)
    t = [math.pi * pa / (na + 1) for na, pa in zip(n, p)]
    S, M = symbols(ndim, t)
    lr = S / h ** 2 - (omega / cval) ** 2 * M
    li = omega * Rval * M
    w, dt, a, b = o.omega_c, o.dt, o.alpha, o.beta
    th = w * dt
    Kp = dt ** 2 / a * (lr + w ** 2) - dt * b * (1 - math.cos(th)) / a * (li / w)
    Lp = b * dt / a * (li / w)
    for T, rho in ((3, 0.25), (5, 0.0)):
        Ns = T * o.nP
        rr = rho if rho > 0 else 1.0 / T
        s, sm = 0j, 0j
        for j in range(Ns):
            fj = oracle.window(1 - j / Ns, rr) * np.exp(2j * math.pi * j / o.nP)
            s, sm = (2 - Kp - Lp) * s - (1 - Lp) * sm + dt ** 2 / a * fj, s
        U = o.precond(e.astype(np.complex128), T, rho, variant=1)
        assert np.linalg.norm(U - s * e) <= 1e-12 * abs(s) * np.linalg.norm(e)


def test_abd_converges_to_inverse_and_gmres_matches_lu():
    """Sec. 6.2 (convergence theorem): S_T^abd F -> H^-1 F as T grows; GMRES
    preconditioned by S_T^abd reaches the sparse-LU solution."""
    p, R = problem((14, 12), 90)
    R = R + 0.5 * p.omega                        # uniform floor: a spectral gap
    o = oracle.Op(p.n, p.h, p.omega, p.c, R, damping="cell")
    H = oracle.assemble_H(p.n, p.h, p.omega, p.c, R, damping="cell")
    U = spla.spsolve(H.tocsc(), p.F.reshape(-1)).reshape(p.n)
    errs = [np.linalg.norm(o.precond(p.F, T, 0.25, variant=1) - U) / np.linalg.norm(U)
            for T in (2, 4, 8, 16, 32)]
    assert all(b < a for a, b in zip(errs, errs[1:])) and errs[-1] < 1e-6, errs
    with pytest.raises(oracle.OracleError):
        o.precond(p.F, 4, 0.25, variant=0)      # Table 1 is the I_acd algorithm
    Ug, info = o.gmres(p.F, T=3, tol=1e-10)
    assert info["status"] == 0
    assert np.linalg.norm(Ug - U) <= 1e-8 * np.linalg.norm(U)
