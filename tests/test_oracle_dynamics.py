"""Pins of the oracle's Krylov kernel, forces, integrator and SCF."""

import dataclasses

import numpy as np
import pytest

from synth import carbon_cluster, ModelParams
from oracle import model, density, krylov, dynamics


def _jacobian_apply(sys_, X, beta):
    F = model.fock(X, sys_.R, sys_.onecenter, sys_.noise, sys_.params)
    dm = density.density_matrix(F, sys_.n_elec, beta)

    def jac(V):
        F1 = model.two_electron(V, sys_.R, sys_.onecenter, sys_.noise, sys_.params)
        return density.response(F, F1, sys_.n_elec, beta, dm) - V
    return dm["P"], jac


def _start_density(sys_, rng):
    n = sys_.n_orb
    X = np.eye(n) * sys_.n_elec / n + 0.05 * rng.standard_normal((n, n))
    return 0.5 * (X + X.T)


def test_full_rank_krylov_equals_exact_inverse_jacobian():
    sys_ = carbon_cluster(2, 8)
    n = sys_.n_orb
    beta = density.beta_of(3000.0)
    X = _start_density(sys_, np.random.default_rng(8))
    P0, jac = _jacobian_apply(sys_, X, beta)
    # J assembled column by column on the orthonormal symmetric basis, solved by LU
    iu = np.triu_indices(n)
    basis = []
    for i, j in zip(*iu):
        E = np.zeros((n, n))
        if i == j:
            E[i, i] = 1.0
        else:
            E[i, j] = E[j, i] = 1.0 / np.sqrt(2.0)
        basis.append(E)
    coords = lambda M: np.array([np.sum(B * M) for B in basis])
    J = np.array([coords(jac(B)) for B in basis]).T
    W0 = P0 - X
    y = np.linalg.solve(J, coords(W0))
    Yref = sum(c * B for c, B in zip(y, basis))
    Y, rank, rel = krylov.krylov_kernel(X, P0, jac, m=len(basis))
    assert rel < 1e-10
    np.testing.assert_allclose(Y, Yref, atol=1e-9 * np.abs(Yref).max())


def _assembled_jacobian(sys_, X, beta):
    """J of the residual on the orthonormal basis of symmetric n x n matrices,
    assembled column by column, with the coordinate maps."""
    n = sys_.n_orb
    P0, jac = _jacobian_apply(sys_, X, beta)
    basis = []
    for i, j in zip(*np.triu_indices(n)):
        E = np.zeros((n, n))
        if i == j:
            E[i, i] = 1.0
        else:
            E[i, j] = E[j, i] = 1.0 / np.sqrt(2.0)
        basis.append(E)
    coords = lambda M: np.array([np.sum(B * M) for B in basis])
    mat = lambda y: sum(c * B for c, B in zip(y, basis))
    J = np.array([coords(jac(B)) for B in basis]).T
    return P0, jac, J, coords, mat


def test_krylov_breaks_down_at_the_grade_of_the_symmetric_space():
    # a 1-atom system: its symmetric 4 x 4 matrices span 10 dimensions, so a
    # rank-16 request must end at rank <= 10 (breakdown), where Y solves
    # J Y = W0 on that space exactly; the basis stays symmetric throughout
    # (W0 = P0 - X carries the rounding asymmetry of P0, which the symmetric
    # responses pass on without growth)
    sys_ = carbon_cluster(1, 21)
    beta = density.beta_of(3000.0)
    X = _start_density(sys_, np.random.default_rng(41))
    P0, jac, J, coords, mat = _assembled_jacobian(sys_, X, beta)
    Yref = mat(np.linalg.solve(J, coords(P0 - X)))
    Y, rank, rel = krylov.krylov_kernel(X, P0, jac, 16)
    assert rank <= 10, rank
    assert rel < 1e-12
    assert np.abs(Y - Y.T).max() <= 1e-14 * np.abs(Y).max()
    np.testing.assert_allclose(Y, Yref, atol=1e-10 * np.abs(Yref).max())


def test_krylov_early_stop_is_the_first_rank_below_tol():
    # Eq. 34 over span{V_1..V_k} = span{W0, J W0, .., J^(k-1) W0} with
    # M = (W^T W)^-1 is the least-squares solution of J Y = W0 over that
    # Krylov space (GMRES).  Reference: the Krylov matrix built by repeated
    # products with the assembled J, orthonormalised by numpy's QR, and the
    # small least-squares problem solved by lstsq.  With tol > 0 the kernel
    # must stop at the first rank whose relative residual is below tol and
    # return that rank's solution.
    sys_ = carbon_cluster(2, 8)
    beta = density.beta_of(3000.0)
    X = _start_density(sys_, np.random.default_rng(8))
    P0, jac, J, coords, mat = _assembled_jacobian(sys_, X, beta)
    w0 = coords(P0 - X)
    cols = [w0 / np.linalg.norm(w0)]
    for _ in range(7):
        v = J @ cols[-1]
        cols.append(v / np.linalg.norm(v))
    res, sols = [], []
    for k in range(1, 8):
        Q, _ = np.linalg.qr(np.array(cols[:k]).T)
        y, *_ = np.linalg.lstsq(J @ Q, w0, rcond=None)
        res.append(np.linalg.norm(J @ Q @ y - w0) / np.linalg.norm(w0))
        sols.append(Q @ y)
    assert all(b < a for a, b in zip(res, res[1:]))   # GMRES residuals decrease
    for k_stop in (2, 3, 5):
        tol = np.sqrt(res[k_stop - 2] * res[k_stop - 1])   # between ranks k_stop - 1 and k_stop
        Y, rank, rel = krylov.krylov_kernel(X, P0, jac, m=7, tol=tol)
        assert rank == k_stop, (k_stop, rank, res)
        assert rel == pytest.approx(res[k_stop - 1], rel=1e-8)
        np.testing.assert_allclose(coords(Y), sols[k_stop - 1], atol=1e-9 * np.abs(sols[k_stop - 1]).max())
    # tol = 0 runs the full requested rank
    Y, rank, rel = krylov.krylov_kernel(X, P0, jac, m=4, tol=0.0)
    assert rank == 4 and rel == pytest.approx(res[3], rel=1e-8)


def test_rank_one_closed_form_and_zero_interaction_limit():
    sys_ = carbon_cluster(3, 9)
    beta = density.beta_of(3000.0)
    X = _start_density(sys_, np.random.default_rng(9))
    P0, jac = _jacobian_apply(sys_, X, beta)
    W0 = P0 - X
    V1 = W0 / np.linalg.norm(W0)
    W1 = jac(V1)
    Y, rank, _ = krylov.krylov_kernel(X, P0, jac, m=1)
    np.testing.assert_allclose(Y, V1 * np.sum(W1 * W0) / np.sum(W1 * W1), atol=1e-13)
    # no two-electron response: J = -I, so the kernel returns -W0 (original XL-BOMD, c = 1)
    Y, rank, rel = krylov.krylov_kernel(X, P0, lambda V: -V, m=3)
    np.testing.assert_allclose(Y, -W0, atol=1e-13)
    assert rank == 1 and rel < 1e-14


def test_forces_match_finite_differences_of_shadow_energy():
    sys_ = carbon_cluster(4, 10)
    st = dynamics.Settings(T_e=3000.0, m=2, dt=0.5)
    X = _start_density(sys_, np.random.default_rng(10))
    ev = dynamics.evaluate(sys_.R, X, sys_, st, with_kernel=False)
    h = 1e-5
    fd = np.zeros_like(sys_.R)
    for i in range(sys_.n_atoms):
        for k in range(3):
            Rp, Rm = sys_.R.copy(), sys_.R.copy()
            Rp[i, k] += h
            Rm[i, k] -= h
            Up = dynamics.evaluate(Rp, X, sys_, st, with_kernel=False)["U"]
            Um = dynamics.evaluate(Rm, X, sys_, st, with_kernel=False)["U"]
            fd[i, k] = -(Up - Um) / (2 * h)
    np.testing.assert_allclose(ev["forces"], fd, atol=2e-6 * max(1.0, np.abs(fd).max()))
    np.testing.assert_allclose(ev["forces"].sum(0), 0.0, atol=1e-10)


def test_entropy_factor_two_is_the_stationary_one():
    # With -T_e S instead of -2 T_e S the forces at fixed X would miss a term:
    # the FD gradient of that alternative energy disagrees with eq. 37's forces.
    sys_ = carbon_cluster(3, 12)
    st = dynamics.Settings(T_e=8000.0, m=2, dt=0.5)
    X = _start_density(sys_, np.random.default_rng(12))
    ev = dynamics.evaluate(sys_.R, X, sys_, st, with_kernel=False)
    h = 1e-5

    def u_alt(R):
        e = dynamics.evaluate(R, X, sys_, st, with_kernel=False)
        return e["U"] + e["S"] / st.beta
    Rp, Rm = sys_.R.copy(), sys_.R.copy()
    Rp[0, 0] += h
    Rm[0, 0] -= h
    fd_alt = -(u_alt(Rp) - u_alt(Rm)) / (2 * h)
    assert abs(fd_alt - ev["forces"][0, 0]) > 1e-4


def test_energy_fluctuation_scales_as_dt_squared():
    sys_ = carbon_cluster(6, 13)
    st0 = dynamics.Settings(T_e=3000.0, m=3, dt=0.2)
    Xmin = dynamics.scf(sys_, st0, m=30)
    spans = []
    for dt in (0.2, 0.1):
        st = dataclasses.replace(st0, dt=dt)
        s = dynamics.init_state(sys_, st, Xmin)
        E = []
        for _ in range(int(round(2.0 / dt))):
            s, rep = dynamics.md_step(s, sys_, st)
            E.append(rep["E_tot"])
        spans.append(np.ptp(E))
    ratio = spans[0] / spans[1]
    assert 3.0 < ratio < 5.5, ratio


def test_integration_is_time_reversible_without_damping():
    sys_ = carbon_cluster(5, 14)
    st = dynamics.Settings(T_e=3000.0, m=3, dt=0.2, alpha=0.0)
    rng = np.random.default_rng(14)
    X0 = _start_density(sys_, rng)
    s = dynamics.init_state(sys_, st, X0)
    s.Xhist[1] = s.Xhist[0] + 0.001 * (s.Xhist[0] - X0.T)
    start = (s.R.copy(), s.Xhist[0].copy())
    for _ in range(5):
        s, _ = dynamics.md_step(s, sys_, st)
    # reverse: flip the velocities; the backward X step from X(t) needs the
    # history (X(t), X(t+dt)) with X(t+dt) the forward prediction of eq. 35
    Xnext = dynamics.integrate_x(s.Xhist, s.Y, st)
    back = dynamics.MDState(R=s.R, V=-s.V, A=s.A, Xhist=[s.Xhist[0], Xnext] + s.Xhist[2:],
                            Y=s.Y, mu=s.mu)
    for _ in range(5):
        back, _ = dynamics.md_step(back, sys_, st)
    np.testing.assert_allclose(back.R, start[0], atol=1e-9)
    np.testing.assert_allclose(back.Xhist[0], start[1], atol=1e-9)


def test_damping_coefficients_are_consistent():
    # the damping sum of eq. 35 vanishes on polynomial histories of degree 1
    # and on the cubic term (sum c_k = sum k c_k = sum k^3 c_k = 0), so it
    # leaves a smoothly moving X(t) alone up to its high-order content
    c = np.array(dynamics.XL_C)
    k = np.arange(7)
    assert c.sum() == 0.0 and (k * c).sum() == 0.0 and (k**3 * c).sum() == 0.0


def _error_rate(Xhist0, st, steps):
    """Iterate the oracle's eq. 35 update on a 1 x 1 'density' with ground
    state X_min = 0 and an exact kernel.  Near X_min the residual is
    W0 = D0[X] - X = J (X - X_min), so Y = J^-1 W0 = X - X_min = X.  Returns
    the asymptotic factor per step by which the history's norm changes."""
    hist = [np.array([[x]]) for x in Xhist0]
    errs = []
    for _ in range(steps):
        Y = hist[0]
        Xn = dynamics.integrate_x(hist, Y, st)
        hist = [Xn] + hist[:-1]
        errs.append(np.sqrt(sum(float(h[0, 0]) ** 2 for h in hist)))
    a, b = steps // 2, steps - 1
    return (errs[b] / errs[a]) ** (1.0 / (b - a))


def test_damping_alpha_makes_the_electronic_recurrence_contract():
    # Linearised about the ground state X_min = 0 with an exact kernel, eq. 35
    # becomes e_{n+1} = (2 - kappa) e_n - e_{n-1} + alpha sum_k c_k e_{n-k}.
    # Without damping (alpha = 0) it is the Verlet oscillator, |z| = 1 for
    # 0 < kappa < 4: errors neither grow nor decay.  The damping the method's
    # coefficients were chosen for contracts every mode, weakly (spectral
    # radius just below one); an alpha ten times larger, or the damping sum
    # with its sign flipped, makes the recurrence blow up.  Both the oracle's
    # integrator and its constants enter through integrate_x.
    rng = np.random.default_rng(35)
    h0 = list(rng.standard_normal(7))
    base = dynamics.Settings(T_e=3000.0, m=0, dt=0.5)
    r_tab = _error_rate(h0, base, 2000)
    r_undamped = _error_rate(h0, dataclasses.replace(base, alpha=0.0), 2000)
    r_big = _error_rate(h0, dataclasses.replace(base, alpha=10 * base.alpha), 400)
    r_flip = _error_rate(h0, dataclasses.replace(base, c=tuple(-x for x in base.c)), 2000)
    assert abs(r_undamped - 1.0) < 2e-3, r_undamped
    assert 0.90 < r_tab < 0.99, r_tab
    assert r_big > 1.2, r_big
    assert r_flip > 1.0, r_flip


def test_scf_reaches_fixed_point():
    sys_ = carbon_cluster(5, 15)
    st = dynamics.Settings(T_e=3000.0, m=3, dt=0.5)
    X = dynamics.scf(sys_, st, m=30, tol=1e-10)
    F = model.fock(X, sys_.R, sys_.onecenter, sys_.noise, sys_.params)
    P = density.density_matrix(F, sys_.n_elec, st.beta)["P"]
    assert np.linalg.norm(P - X) < 1e-9


def test_original_kernel_is_scaled_identity():
    # m = 0 is the original XL-BOMD kernel K = -c I: eq. 35's kernel term
    # becomes -c (P0 - X).  Its sign convention is the Krylov kernel's: with
    # a vanishing response (J = -I) the full-rank Krylov kernel J^-1 W0 is
    # exactly the c = 1 scaled identity.
    sys_ = carbon_cluster(4, 21)
    rng = np.random.default_rng(21)
    X = _start_density(sys_, rng)
    st = dynamics.Settings(T_e=3000.0, m=0, dt=0.5, kernel_c=0.9)
    ev = dynamics.evaluate(sys_.R, X, sys_, st)
    W0 = ev["P0"] - X
    np.testing.assert_array_equal(ev["Y"], -0.9 * W0)
    assert ev["rank"] == 0 and ev["relres"] == 1.0
    Y, rank, rel = krylov.krylov_kernel(X, ev["P0"], lambda V: -V, 3)
    assert rank == 1 and rel < 1e-14
    np.testing.assert_allclose(Y, -W0, rtol=0, atol=1e-14 * np.abs(W0).max())


def test_original_xlbomd_unstable_where_ksa_is_stable():
    # Results, low-gap fullerene test: with strong charge response the
    # scaled-identity kernel (c = 1) lets the electronic residual grow without
    # bound, a smaller c keeps it bounded but less tight, and the rank-3 KSA
    # kernel stays stable and tight.  Here on the 6-atom cluster, 20 steps of
    # 0.1 fs from the ground state.
    import dataclasses
    sys_ = carbon_cluster(6, 13)
    st0 = dynamics.Settings(T_e=3000.0, m=3, dt=0.1)
    Xmin = dynamics.scf(sys_, st0, m=30)
    res = {}
    for m, c in ((3, 1.0), (0, 1.0), (0, 0.5)):
        st = dataclasses.replace(st0, m=m, kernel_c=c)
        s = dynamics.init_state(sys_, st, Xmin)
        E, W = [], []
        for _ in range(20):
            s, rep = dynamics.md_step(s, sys_, st)
            E.append(rep["E_tot"])
            W.append(rep["W0"])
        res[(m, c)] = (np.ptp(E), max(W))
    ksa, xl1, xl05 = res[(3, 1.0)], res[(0, 1.0)], res[(0, 0.5)]
    assert ksa[0] < 1e-2 and ksa[1] < 2e-3
    assert xl1[1] > 100 * ksa[1] and xl1[0] > 1.0
    assert xl05[1] < 1e-2 and xl05[1] > ksa[1]


def test_langevin_without_friction_is_the_nve_step():
    # gamma = 0: the Ornstein-Uhlenbeck update is the identity and BAOAB's two
    # half drifts make the leapfrog drift of md_step
    sys_ = carbon_cluster(5, 14)
    st = dynamics.Settings(T_e=3000.0, m=3, dt=0.2)
    rng = np.random.default_rng(3)
    s0 = dynamics.init_state(sys_, st, _start_density(sys_, rng))
    s0.V = 0.01 * rng.standard_normal(s0.R.shape)
    a, ra = dynamics.md_step(s0, sys_, st)
    b, rb = dynamics.langevin_step(s0, sys_, st, 0.0, 300.0, rng.standard_normal(s0.R.shape))
    np.testing.assert_allclose(b.R, a.R, rtol=0, atol=1e-14)
    np.testing.assert_allclose(b.V, a.V, rtol=0, atol=1e-13)
    np.testing.assert_array_equal(b.Xhist[0], a.Xhist[0])
    assert rb["E_tot"] == pytest.approx(ra["E_tot"], rel=1e-13)


def test_ou_update_keeps_the_maxwell_boltzmann_variance():
    # equipartition: (1/2) M <v^2> = (1/2) k_B T per Cartesian component, and
    # the exact Ornstein-Uhlenbeck step maps that distribution onto itself
    mass, T, dt = 12.011, 300.0, 0.5
    var = density.KB_EV_PER_K * T / mass * dynamics.EV_PER_AMU_TO_A2_PER_FS2
    rng = np.random.default_rng(11)
    v = np.sqrt(var) * rng.standard_normal(400_000)
    for gamma in (0.01, 0.2, 5.0):
        c1, c2 = dynamics.ou_coefficients(gamma, T, dt, mass)
        w = c1 * v + c2 * rng.standard_normal(v.size)
        assert abs(w.var() / var - 1.0) < 0.012
        assert abs(w.mean()) < 0.01 * np.sqrt(var)


def test_langevin_thermalises_to_the_bath_temperature():
    # a 4-atom cluster started far from equilibrium: after the transient the
    # mean kinetic energy is (3N/2) k_B T (statistical error ~6% here)
    sys_ = carbon_cluster(4, 31)
    st = dynamics.Settings(T_e=3000.0, m=2, dt=0.25)
    s = dynamics.init_state(sys_, st, dynamics.scf(sys_, st, m=20))
    rng = np.random.default_rng(5)
    KE = []
    for _ in range(1600):
        s, rep = dynamics.langevin_step(s, sys_, st, 0.1, 300.0, rng.standard_normal((sys_.n_atoms, 3)))
        KE.append(rep["KE"])
    ratio = np.mean(KE[400:]) / (1.5 * sys_.n_atoms * density.KB_EV_PER_K * 300.0)
    assert abs(ratio - 1.0) < 0.15, ratio
