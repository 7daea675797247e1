"""Pins of the oracle's per-node pieces against facts the paper and the
mathematics fix (no GPU). Each test would fail on a plausible slip: a wrong
weight, sign, index, opposite direction or forcing prefactor."""
import math

import numpy as np
import pytest

RNG = np.random.Generator(np.random.PCG64(1234))


def _rand_state(n=20):
    for _ in range(n):
        rho = 1.0 + 0.2 * RNG.uniform(-1, 1)
        u = 0.1 * RNG.uniform(-1, 1, size=2)
        F = 1e-3 * RNG.uniform(-1, 1, size=2)
        yield rho, u, F


def test_lattice_matches_eq_d2q9(oracle):
    """Velocities follow the angle formula of eq. (D2Q9); opposite map is e_{-a} = -e_a
    (Sec. 2.1: f_{-1} = f_3, f_{-0} = f_0); weights 4/9, 1/9, 1/36 (eq. feq)."""
    ex, ey, w, opp = oracle.lattice()
    for a in range(1, 5):
        t = (a - 1) * math.pi / 2
        assert (ex[a], ey[a]) == (round(math.cos(t)), round(math.sin(t)))
    for a in range(5, 9):
        t = (2 * a - 9) * math.pi / 4
        assert (ex[a], ey[a]) == (round(math.sqrt(2) * math.cos(t)), round(math.sqrt(2) * math.sin(t)))
    assert (ex[0], ey[0]) == (0, 0)
    assert opp[1] == 3 and opp[0] == 0
    for a in range(9):
        assert ex[opp[a]] == -ex[a] and ey[opp[a]] == -ey[a]
    assert np.allclose(w, [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4, rtol=0, atol=1e-17)


def test_t1_equilibrium_moments(oracle):
    """T1: sum f^eq = rho, sum e f^eq = rho u, sum e e f^eq = rho/3 I + rho u u;
    sum w = 1, sum w e e = I/3 (eq. feq with c_s^2 = 1/3)."""
    ex, ey, w, _ = oracle.lattice()
    e = np.stack([ex, ey], 1).astype(float)
    assert abs(w.sum() - 1) < 1e-15
    assert np.allclose(np.einsum("a,ai,aj->ij", w, e, e), np.eye(2) / 3, atol=1e-16)
    for rho, u, _ in _rand_state():
        f = oracle.feq(rho, u[0], u[1])
        assert abs(f.sum() - rho) < 1e-15 * rho
        assert np.allclose(e.T @ f, rho * u, rtol=0, atol=1e-16)
        pi = np.einsum("a,ai,aj->ij", f, e, e)
        assert np.allclose(pi, rho / 3 * np.eye(2) + rho * np.outer(u, u), rtol=0, atol=2e-16)


def test_t2_guo_moments(oracle):
    """T2: the forcing term (eq. external-force-term) has sum F_a = 0,
    sum e F_a = F, sum e e F_a = u F + F u, and antisymmetric part 3 w e.F."""
    ex, ey, w, opp = oracle.lattice()
    e = np.stack([ex, ey], 1).astype(float)
    for _, u, F in _rand_state():
        Fa = oracle.guo(u[0], u[1], F[0], F[1])
        assert abs(Fa.sum()) < 1e-18
        assert np.allclose(e.T @ Fa, F, rtol=0, atol=1e-18)
        m2 = np.einsum("a,ai,aj->ij", Fa, e, e)
        assert np.allclose(m2, np.outer(u, F) + np.outer(F, u), rtol=0, atol=1e-18)
        anti = 0.5 * (Fa - Fa[opp])
        assert np.allclose(anti, 3 * w * (e @ F), rtol=0, atol=1e-18)


@pytest.mark.parametrize("chi", [0, 1])
def test_t3_collision_invariants(oracle, chi):
    """T3: mass is unchanged by the collision and momentum gains exactly the total
    force F = F_b + F_VP (eqs. rho*velocity-ex and collision-modified)."""
    ex, ey, w, _ = oracle.lattice()
    e = np.stack([ex, ey], 1).astype(float)
    tau_s = 0.7
    tau_a = oracle.tau_minus(tau_s, 0.25)
    for rho, u, fb in _rand_state():
        f = oracle.feq(rho, u[0], u[1]) + 1e-3 * RNG.uniform(-1, 1, 9)
        uo = 0.05 * RNG.uniform(-1, 1, 2)
        g, fl = oracle.collide_node(f, tau_s, tau_a, 1e-4, chi, uo, fb)
        assert abs(g.sum() - f.sum()) < 2e-15
        F = fb + fl[3:5]
        assert np.allclose(e.T @ g, e.T @ f + F, rtol=0, atol=1e-15 * (1 + np.abs(F).max()))
        if chi == 0:
            assert np.all(fl[3:5] == 0.0)


def test_tau_minus_magic_parameter(oracle):
    """Lambda = (tau_s - 1/2)(tau_a - 1/2) (Sec. 2.1)."""
    for ts, lam in [(0.8, 0.25), (0.56, 3 / 16), (1.7, 0.1)]:
        ta = oracle.tau_minus(ts, lam)
        assert abs((ts - 0.5) * (ta - 0.5) - lam) < 1e-15
    assert abs(oracle.tau_minus(0.56, 3 / 16) - 3.625) < 1e-13


def test_t5_srt_special_case(oracle):
    """T5: with Lambda = (tau - 1/2)^2 the two times coincide and the step is the
    single-relaxation BGK step with Guo forcing, g = f - (f - f^eq)/tau + (1 - 1/2tau) F_a.
    The BGK step is restated here from its textbook form."""
    ex, ey, w, _ = oracle.lattice()
    e = np.stack([ex, ey], 1).astype(float)
    tau = 0.83
    tau_a = oracle.tau_minus(tau, (tau - 0.5) ** 2)
    assert abs(tau_a - tau) < 1e-15
    for rho, u, fb in _rand_state():
        f = oracle.feq(rho, u[0], u[1]) + 1e-3 * RNG.uniform(-1, 1, 9)
        g, fl = oracle.collide_node(f, tau, tau_a, 1e-4, 0, (0.0, 0.0), fb)
        r = f.sum()
        vel = (e.T @ f + 0.5 * fb) / r
        eu = e @ vel
        feq = w * r * (1 + 3 * eu + 4.5 * eu ** 2 - 1.5 * vel @ vel)
        Fa = w * (3 * (e - vel) @ fb + 9 * eu * (e @ fb))
        bgk = f - (f - feq) / tau + (1 - 0.5 / tau) * Fa
        assert np.allclose(g, bgk, rtol=0, atol=1e-15)


def test_t6_t7_vp_closed_forms(oracle):
    """T6: F_VP + (chi rho / eta)(u* + du - U_O) = 0 (eqs. VP-force-1, d-V,
    force-density). T7: in a solid node |u - U_O| = 2 eta/(2 eta + 1) |u* - U_O|.
    Also du = F_VP/(2 rho) (eq. rho*delta-velocity)."""
    for eta in (1e-2, 1e-4, 1e-8):
        for rho, u, _ in _rand_state():
            uo = 0.05 * RNG.uniform(-1, 1, 2)
            dux, duy, fx, fy = oracle.vp(rho, u[0], u[1], 1, uo[0], uo[1], eta)
            F = np.array([fx, fy])
            du = np.array([dux, duy])
            resid = F + rho / eta * (u + du - uo)
            # the residual is evaluated in FP64: u* + du - U_O cancels to ~2 eta |u* - U_O|,
            # so its rounding (a few ulps of |u|) is amplified by rho/eta
            ulp_bound = 8 * 2.2e-16 * (np.abs(u).max() + np.abs(du).max() + np.abs(uo).max()) * rho / eta
            assert np.abs(resid).max() <= 1e-14 * np.abs(F).max() + ulp_bound
            ratio = np.linalg.norm(u + du - uo) / np.linalg.norm(u - uo)
            assert abs(ratio - 2 * eta / (2 * eta + 1)) <= 1e-14 * max(1.0, 2 * eta / (2 * eta + 1)) + 1e-12 * eta
            assert np.allclose(du, F / (2 * rho), rtol=1e-15, atol=0)
            z = oracle.vp(rho, u[0], u[1], 0, uo[0], uo[1], eta)
            assert np.all(z == 0.0)
