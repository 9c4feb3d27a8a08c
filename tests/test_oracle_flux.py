"""Pins for the numerical fluxes (Sec. 2.3: Roe and local Lax-Friedrichs).

Invariants any correct implementation satisfies: consistency with the
physical flux, conservation (antisymmetry in the two states and the
normal), rotation invariance, pure upwinding of the Roe flux for
supersonic states (equivalent to the Roe property F+ - F- = A~ (w+ - w-)),
the LLF speed equal to the spectral radius of the flux Jacobian (computed
numerically here), and zero mass flux through a land boundary.
"""
import numpy as np
import pytest

from oracle import physics

G, H0 = 9.81, 1e-3


def rand_states(rng, n, hb):
    zeta = rng.uniform(-0.5, 0.5, n)
    q = rng.normal(0, 2.0, (2, n))
    return np.stack([zeta, q[0], q[1]])


@pytest.mark.parametrize("kind", ["roe", "llf"])
def test_consistency(kind):
    rng = np.random.default_rng(0)
    hb = rng.uniform(1, 30, 50)
    w = rand_states(rng, 50, hb)
    th = rng.uniform(0, 2 * np.pi, 50)
    nx, ny = np.cos(th), np.sin(th)
    F = physics.numerical_flux(kind, w, w, hb, nx, ny, G, H0)
    Fn = physics.flux_n(w[0], w[1], w[2], hb, nx, ny, G, H0)
    np.testing.assert_allclose(F, Fn, rtol=1e-14, atol=1e-12)


@pytest.mark.parametrize("kind", ["roe", "llf"])
def test_conservation_antisymmetry(kind):
    rng = np.random.default_rng(1)
    hb = rng.uniform(1, 30, 50)
    a, b = rand_states(rng, 50, hb), rand_states(rng, 50, hb)
    th = rng.uniform(0, 2 * np.pi, 50)
    nx, ny = np.cos(th), np.sin(th)
    F1 = physics.numerical_flux(kind, a, b, hb, nx, ny, G, H0)
    F2 = physics.numerical_flux(kind, b, a, hb, -nx, -ny, G, H0)
    np.testing.assert_allclose(F1, -F2, rtol=1e-13, atol=1e-11)


@pytest.mark.parametrize("kind", ["roe", "llf"])
def test_rotation_invariance(kind):
    rng = np.random.default_rng(2)
    hb = rng.uniform(1, 30, 40)
    a, b = rand_states(rng, 40, hb), rand_states(rng, 40, hb)
    th = rng.uniform(0, 2 * np.pi, 40)
    nx, ny = np.cos(th), np.sin(th)
    F = physics.numerical_flux(kind, a, b, hb, nx, ny, G, H0)
    phi = 0.7
    c, s = np.cos(phi), np.sin(phi)
    rot = lambda w: np.stack([w[0], c * w[1] - s * w[2], s * w[1] + c * w[2]])  # noqa: E731
    Fr = physics.numerical_flux(kind, rot(a), rot(b), hb, c * nx - s * ny, s * nx + c * ny, G, H0)
    np.testing.assert_allclose(Fr, rot(F), rtol=1e-12, atol=1e-10)


def test_roe_supersonic_is_pure_upwind():
    # with every Roe wave speed of one sign the Roe flux is the upwind
    # physical flux exactly when the Roe property holds
    rng = np.random.default_rng(3)
    n = 40
    hb = rng.uniform(0.5, 2.0, n)
    H_l = hb + rng.uniform(-0.1, 0.1, n); H_r = hb + rng.uniform(-0.1, 0.1, n)
    u_l = rng.uniform(8, 12, n); u_r = rng.uniform(8, 12, n)     # > sqrt(g H) ~ 4.5
    v_l = rng.normal(0, 1, n); v_r = rng.normal(0, 1, n)
    wl = np.stack([H_l - hb, H_l * u_l, H_l * v_l]); wr = np.stack([H_r - hb, H_r * u_r, H_r * v_r])
    one, zero = np.ones(n), np.zeros(n)
    F = physics.roe(wl, wr, hb, one, zero, G, H0)
    np.testing.assert_allclose(F, physics.flux_n(*wl, hb, one, zero, G, H0), rtol=1e-12, atol=1e-11)
    F = physics.roe(wr, wl, hb, -one, zero, G, H0)      # flow against the normal: upwind is the right state
    np.testing.assert_allclose(F, physics.flux_n(*wl, hb, -one, zero, G, H0), rtol=1e-12, atol=1e-11)


def test_llf_speed_is_spectral_radius():
    rng = np.random.default_rng(4)
    for _ in range(20):
        hb = np.array([rng.uniform(1, 20)])
        a = rand_states(rng, 1, hb); b = rand_states(rng, 1, hb)
        th = rng.uniform(0, 2 * np.pi); nx, ny = np.array([np.cos(th)]), np.array([np.sin(th)])

        def jac(w):
            eps = 1e-6
            J = np.zeros((3, 3))
            for k in range(3):
                d = np.zeros((3, 1)); d[k] = eps
                J[:, k] = ((physics.flux_n(*(w + d), hb, nx, ny, G, H0)
                            - physics.flux_n(*(w - d), hb, nx, ny, G, H0)) / (2 * eps))[:, 0]
            return J
        rho = max(np.abs(np.linalg.eigvals(jac(a))).max(), np.abs(np.linalg.eigvals(jac(b))).max())
        F = physics.llf(a, b, hb, nx, ny, G, H0)
        central = 0.5 * (physics.flux_n(*a, hb, nx, ny, G, H0) + physics.flux_n(*b, hb, nx, ny, G, H0))
        lam = -2.0 * (F - central) / (b - a)
        np.testing.assert_allclose(lam[:, 0], rho, rtol=1e-6)


@pytest.mark.parametrize("kind", ["roe", "llf"])
def test_land_mirror_has_zero_mass_flux_and_lake_at_rest_is_hydrostatic(kind):
    rng = np.random.default_rng(5)
    hb = rng.uniform(0.5, 30, 60)
    w = rand_states(rng, 60, hb)
    th = rng.uniform(0, 2 * np.pi, 60)
    nx, ny = np.cos(th), np.sin(th)
    qn = w[1] * nx + w[2] * ny
    mirror = np.stack([w[0], w[1] - 2 * qn * nx, w[2] - 2 * qn * ny])
    F = physics.numerical_flux(kind, w, mirror, hb, nx, ny, G, H0)
    assert np.max(np.abs(F[0])) < 1e-13
    rest = np.stack([w[0], 0 * w[0], 0 * w[0]])
    F = physics.numerical_flux(kind, rest, rest.copy(), hb, nx, ny, G, H0)
    P = 0.5 * G * (((w[0] + hb) ** 2) - hb ** 2)
    np.testing.assert_allclose(F[1], P * nx, rtol=1e-12, atol=1e-9)
    np.testing.assert_allclose(F[2], P * ny, rtol=1e-12, atol=1e-9)
    assert np.all(F[0] == 0)
