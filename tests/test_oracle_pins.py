"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a brute-force
sum, a closed form, an invariant, a textbook identity or a finite difference.
"""

import math

import numpy as np
import pytest

import oracle as O
from oracle import dft, model, adjoint, precond, optim, fields, ensemble
from oracle.model import Physics, Obs


# ---------------------------------------------------------------- DFT -----

def brute_dft2(f):
    """O(N^4) double loop with math.cos / math.sin of the raw angle."""
    N = f.shape[0]
    out = np.zeros((N, N), dtype=np.complex128)
    for q in range(N):
        for p in range(N):
            acc = 0j
            for j in range(N):
                for i in range(N):
                    ang = -2.0 * math.pi * (p * i + q * j) / N
                    acc += f[j, i] * complex(math.cos(ang), math.sin(ang))
            out[q, p] = acc
    return out


@pytest.mark.parametrize("N", [8, 16])
def test_dft_matches_brute_force(N):
    rng = np.random.default_rng(N)
    f = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    ref = brute_dft2(f)
    got = dft.fft2(f)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-14
    back = dft.ifft2(got)
    assert np.linalg.norm(back - f) / np.linalg.norm(f) < 1e-14


@pytest.mark.parametrize("N", [8, 32, 256])
def test_dft_single_mode_is_delta(N):
    x = 2 * np.pi * np.arange(N) / N
    p, q = 3 % N, (N - 2) % N          # kx = 3, ky = -2
    f = np.exp(1j * (3 * x[None, :] - 2 * x[:, None]))
    F = dft.fft2(f)
    expect = np.zeros((N, N), dtype=np.complex128)
    expect[q, p] = N * N
    assert np.max(np.abs(F - expect)) < 1e-12 * N * N


def test_twiddles_exact_symmetries():
    c, s = dft.twiddles(64)
    assert c[16] == 0.0 and s[16] == 1.0 and c[32] == -1.0 and s[32] == 0.0
    assert np.max(np.abs(c ** 2 + s ** 2 - 1)) < 3e-16
    ref_c = np.array([math.cos(2 * math.pi * m / 64) for m in range(64)])
    assert np.max(np.abs(c - ref_c)) < 1e-15


# ---------------------------------------------------------- operators -----

def test_operators_on_trig_polynomial():
    N = 32
    g = model.grid(N)
    X, Y = np.meshgrid(g.x, g.y)          # X[j][i] = x_i, Y[j][i] = y_j
    m, n = 3, 2
    f = np.sin(m * X) * np.cos(n * Y)
    k2 = m * m + n * n
    assert np.max(np.abs(g.apply(g.m_dx, f) - m * np.cos(m * X) * np.cos(n * Y))) < 1e-13
    assert np.max(np.abs(g.apply(g.m_dy, f) + n * np.sin(m * X) * np.sin(n * Y))) < 1e-13
    assert np.max(np.abs(g.apply(g.m_psi, f) - f / k2)) < 1e-14
    # u = d_y psi, v = -d_x psi with -Lap psi = omega
    assert np.max(np.abs(g.apply(g.m_u, f) + (n / k2) * np.sin(m * X) * np.sin(n * Y))) < 1e-14
    assert np.max(np.abs(g.apply(g.m_v, f) + (m / k2) * np.cos(m * X) * np.cos(n * Y))) < 1e-14
    # P removes the mean and modes outside the 2/3 band
    hi = np.cos(11 * X)                    # Kc = 10 at N = 32
    assert np.max(np.abs(g.apply(g.mask, hi + 5.0))) < 1e-13


def test_band_limit_values():
    for N, Kc in [(64, 21), (128, 42), (256, 85), (512, 170), (1024, 341)]:
        assert (N - 1) // 3 == Kc
        assert N - 2 * Kc > Kc            # de-aliasing: aliased modes land outside S


# ----------------------------------------------------------- forward -----

def test_taylor_green_decay_exact():
    N, k, nu, mu, dt, steps = 32, 2, 1e-2, 0.05, 1e-3, 1000
    ph = Physics(N=N, nu=nu, dt=dt, mu=mu)
    g = model.grid(N)
    X, Y = np.meshgrid(g.x, g.y)
    w0 = 2 * k * k * np.sin(k * X) * np.sin(k * Y)
    wT, _, _ = O.forward(w0, ph, steps)
    expect = w0 * math.exp(-(2 * nu * k * k + mu) * dt * steps)
    assert np.linalg.norm(wT - expect) / np.linalg.norm(expect) < 1e-13


def test_kolmogorov_laminar_closed_form():
    # From rest the nonlinear term vanishes identically (u = U(y), omega = omega(y)),
    # so each mode follows w_{n+1} = E w_n + (h/6)(E + 4 E^{1/2} + 1) F exactly.
    N, nu, mu, A, nf, h, steps = 32, 1.0 / 40, 0.1, 1.0, 4, 1e-3, 400
    ph = Physics(N=N, nu=nu, dt=h, mu=mu, forcing_amp=A, forcing_k=nf)
    g = model.grid(N)
    lam = nu * nf * nf + mu
    E = math.exp(-lam * h)
    E2 = math.exp(-lam * h / 2)
    Y = np.broadcast_to(g.y[:, None], (N, N))
    F = -A * nf * np.cos(nf * Y)               # forcing in vorticity
    w_star = (h / 6) * (E + 4 * E2 + 1) * F / (1 - E)
    wT, _, _ = O.forward(np.zeros((N, N)), ph, steps)
    expect = w_star * (1 - E ** steps)
    assert np.max(np.abs(wT - expect)) < 1e-12 * np.max(np.abs(expect))
    # the discrete fixed point agrees with the laminar state -8 cos 4y
    ws = -A * nf * np.cos(nf * Y) / lam
    assert np.max(np.abs(ws + 8 * np.cos(4 * Y))) < 1e-12
    assert np.max(np.abs(w_star - ws)) < 1e-12 * 8


def _energy_enstrophy(g, w):
    u = g.apply(g.m_u, w)
    v = g.apply(g.m_v, w)
    return 0.5 * np.mean(u * u + v * v), 0.5 * np.mean(w * w)


def test_inviscid_conservation_and_order():
    # The Galerkin-truncated (2/3 mask) nu = mu = 0 dynamics conserves energy and
    # enstrophy exactly (the triple products are alias-free since 3 Kc < N), so the
    # only drift is the time scheme's.  RK4 conserves quadratic invariants to
    # at least order 4; its stability function on the imaginary axis has
    # |R(iy)|^2 = 1 - y^6/72 + O(y^8), so the observed global order is 5.
    N = 32
    g = model.grid(N)
    w0 = O.init_field(N, [3], kind=0, k0=3.0)[0]
    E0, Z0 = _energy_enstrophy(g, w0)
    dz = []
    for h, steps in [(4e-2, 25), (2e-2, 50), (1e-2, 100)]:
        wT, _, _ = O.forward(w0, Physics(N=N, nu=0.0, dt=h), steps)
        _E1, Z1 = _energy_enstrophy(g, wT)
        dz.append(abs(Z1 - Z0) / Z0)
    for a, b in zip(dz[:-1], dz[1:]):
        order = math.log2(a / b)
        assert 3.8 < order < 5.5, order
    wT, _, _ = O.forward(w0, Physics(N=N, nu=0.0, dt=1e-3), 1000)
    E1, Z1 = _energy_enstrophy(g, wT)
    assert abs(E1 - E0) / E0 < 1e-10 and abs(Z1 - Z0) / Z0 < 1e-10


def test_observation_operator_closed_form():
    N, s = 32, 4
    g = model.grid(N)
    X, Y = np.meshgrid(g.x, g.y)
    w = np.cos(3 * X + 2 * Y)                  # psi = w / 13
    u_ex = -(2.0 / 13) * np.sin(3 * X + 2 * Y)
    v_ex = (3.0 / 13) * np.sin(3 * X + 2 * Y)
    o = model.observe(g, g.mask * dft.fft2(w), s)
    assert np.max(np.abs(o[0] - u_ex[::s, ::s])) < 1e-14
    assert np.max(np.abs(o[1] - v_ex[::s, ::s])) < 1e-14


# ----------------------------------------------------------- adjoint -----

@pytest.mark.parametrize("steps", [1, 100])
def test_adjoint_dot_product(steps):
    N = 16
    ph = Physics(N=N, nu=5e-3, dt=5e-3, mu=0.05, forcing_amp=1.0, forcing_k=4)
    rng = np.random.default_rng(steps)
    w0 = O.init_field(N, [11], kind=0, k0=3.0)[0]
    d = rng.standard_normal((N, N))
    m = rng.standard_normal((N, N))
    lhs = float(np.sum(adjoint.tlm_trajectory(w0, d, ph, steps) * m))
    rhs = float(np.sum(d * adjoint.adjoint_trajectory(w0, m, ph, steps)))
    assert abs(lhs - rhs) <= 1e-13 * max(abs(lhs), 1e-300) * 10


def _twin_obs(N, ph, steps, obs_steps, stride, seed):
    truth = O.init_field(N, [seed], kind=0, k0=3.0)[0]
    _, _, mo = O.forward(truth, ph, steps, Obs(stride, obs_steps))
    return Obs(stride, obs_steps, mo)


def test_gradient_central_fd():
    N, steps = 16, 20
    ph = Physics(N=N, nu=1e-2, dt=1e-2)
    obs = _twin_obs(N, ph, steps, [0, 10, 20], 2, seed=5)
    w0 = O.init_field(N, [6], kind=0, k0=3.0)[0]
    J, gr = O.adjoint_gradient(w0, ph, steps, obs)
    assert J > 0
    for seed in range(1000, 1005):
        d = O.init_field(N, [seed], kind=2, target=float(np.sqrt(np.mean(w0 ** 2))))[0]
        eps = 1e-6
        Jp = O.forward(w0 + eps * d, ph, steps, obs)[1]
        Jm = O.forward(w0 - eps * d, ph, steps, obs)[1]
        fd = (Jp - Jm) / (2 * eps)
        ad = float(np.sum(gr * d))
        assert abs(fd - ad) <= 1e-6 * abs(ad), (fd, ad)


def test_gradient_of_exact_observations_is_zero():
    N, steps = 16, 10
    ph = Physics(N=N, nu=1e-2, dt=1e-2)
    truth = O.init_field(N, [2], kind=0, k0=3.0)[0]
    _, _, mo = O.forward(truth, ph, steps, Obs(4, [0, 10]))
    J, gr = O.adjoint_gradient(truth, ph, steps, Obs(4, [0, 10], mo))
    assert J == 0.0 and np.max(np.abs(gr)) == 0.0


def test_horizon_zero_gradient_closed_form():
    # H = 0: J = 1/2 |M U P w - m|^2, so grad = P U^T S^T r (+ V part): compare with FD-free linear algebra
    N, s = 16, 4
    ph = Physics(N=N, nu=1e-2, dt=1e-2)
    g = model.grid(N)
    w = O.init_field(N, [4], kind=0, k0=3.0)[0]
    m = np.zeros((1, 2, N // s, N // s))
    J, gr = O.adjoint_gradient(w, ph, 0, Obs(s, [0], m))
    # J is quadratic in w: J(w) = 1/2 <w, H w>, grad = H w, so <grad, w> = 2 J
    assert abs(float(np.sum(gr * w)) - 2 * J) < 1e-13 * J


# ------------------------------------------------------ precondition -----

def test_precondition_identities():
    N = 32
    g = model.grid(N)
    rng = np.random.default_rng(0)
    f = rng.standard_normal((N, N))
    Pf = g.apply(g.mask, f)
    for kern in [precond.Kernel(0), precond.Kernel(1, 0.1), precond.Kernel(2, 0.5),
                 precond.Kernel(3, 0.01), precond.Kernel(1, 0.05, precond.VORTICITY)]:
        s = O.precondition(f, kern, -0.5)
        back = O.precondition(s, kern, 0.5)
        assert np.linalg.norm(back - Pf) < 1e-12 * np.linalg.norm(Pf)
        full = O.precondition(f, kern, 1.0)
        twice = O.precondition(O.precondition(f, kern, 0.5), kern, 0.5)
        assert np.linalg.norm(full - twice) < 1e-12 * np.linalg.norm(full)


def test_precondition_single_mode_closed_form():
    N = 32
    g = model.grid(N)
    X, Y = np.meshgrid(g.x, g.y)
    f = np.cos(3 * X - 4 * Y)                 # |k| = 5
    for kern, mult in [(precond.Kernel(0), 25.0 ** 0.5),
                       (precond.Kernel(1, 0.1), (25 * math.exp(-0.5)) ** 0.5),
                       (precond.Kernel(2, 0.5), (25 * 5.0 ** -1) ** 0.5),
                       (precond.Kernel(3, 0.02), (25 * math.exp(-0.5)) ** 0.5),
                       (precond.Kernel(2, 0.25, precond.VORTICITY), (5.0 ** -0.5) ** 0.5)]:
        got = O.precondition(f, kern, 0.5)
        assert np.max(np.abs(got - mult * f)) < 1e-13


def test_velocity_metric_parseval_isometry():
    # identity kernel, velocity metric: sum s^2 equals sum |u|^2 (the paper's velocity control)
    N = 32
    g = model.grid(N)
    w = O.init_field(N, [1], kind=0, k0=4.0)[0]
    s = O.precondition(w, precond.Kernel(0), -0.5)
    u = g.apply(g.m_u, w)
    v = g.apply(g.m_v, w)
    assert abs(np.sum(s * s) - np.sum(u * u + v * v)) < 1e-12 * np.sum(u * u + v * v)


def test_vorticity_control_equivalence_appendix_b():
    # W = 1/k^2 under the velocity metric is the identity under the vorticity metric (App. B)
    N = 16
    f = np.random.default_rng(3).standard_normal((N, N))
    a = O.precondition(f, precond.Kernel(2, 1.0, precond.VELOCITY), 0.5)
    b = O.precondition(f, precond.Kernel(0, 0.0, precond.VORTICITY), 0.5)
    assert np.max(np.abs(a - b)) < 1e-15


# ----------------------------------------------------------- optimizer -----

def test_toy_problem_latent_sd():
    # J = 0.01 u_l^2 + u_h^2 with G = diag(100, 1): in s = G^{-1/2} u, J = s_l^2 + s_h^2
    # and grad_s = G^{1/2} grad_u = [2 s_l, 2 s_h] (Sec. II.C).
    Gh = np.array([10.0, 1.0])
    J_u = lambda u: 0.01 * u[0] ** 2 + u[1] ** 2
    grad_u = lambda u: np.array([0.02 * u[0], 2 * u[1]])
    fun = lambda s: J_u(Gh * s)
    fun_grad = lambda s: (J_u(Gh * s), Gh * grad_u(Gh * s))
    s0 = np.array([3.0, -2.0])
    assert np.allclose(fun_grad(s0)[1], 2 * s0)
    x, hist, it, status = optim.minimize(fun_grad, fun, s0, method="sd", max_iter=5)
    # the latent steepest-descent direction points at the minimiser: every Polyak
    # step halves s exactly (J drops by 4 per iteration)
    assert status == 0 and it == 5
    assert np.allclose(x, s0 / 32, rtol=0, atol=1e-15)
    assert np.allclose(hist, [fun(s0) / 4 ** k for k in range(6)], rtol=1e-14)
    # in u itself the same rule zig-zags: the first step is far from the minimiser
    xu, hu, _, _ = optim.minimize(lambda u: (J_u(u), grad_u(u)), J_u, Gh * s0, "sd", 5)
    assert hu[-1] > 10 * hist[-1]


def _dense_bfgs_inverse(pairs, n):
    s, y = pairs[-1]
    H = (np.dot(s, y) / np.dot(y, y)) * np.eye(n)
    for s, y in pairs:
        rho = 1.0 / np.dot(y, s)
        V = np.eye(n) - rho * np.outer(y, s)
        H = V.T @ H @ V + rho * np.outer(s, s)
    return H


def test_two_loop_equals_dense_bfgs():
    rng = np.random.default_rng(7)
    n = 12
    A = rng.standard_normal((n, n))
    A = A @ A.T + n * np.eye(n)
    pairs = []
    for _ in range(5):
        s = rng.standard_normal(n)
        pairs.append((s, A @ s))
    g = rng.standard_normal(n)
    ref = _dense_bfgs_inverse(pairs, n) @ g
    got = optim.lbfgs_two_loop(g, pairs)
    assert np.linalg.norm(got - ref) < 1e-12 * np.linalg.norm(ref)


def test_lbfgs_quadratic_converges_to_solution():
    rng = np.random.default_rng(9)
    n = 20
    Q = rng.standard_normal((n, n))
    A = Q @ Q.T + np.eye(n)
    b = rng.standard_normal(n)
    xs = np.linalg.solve(A, b)
    fun = lambda x: 0.5 * (x - xs) @ A @ (x - xs)      # min J = 0 without cancellation
    fun_grad = lambda x: (fun(x), A @ (x - xs))
    x, hist, it, status = optim.minimize(fun_grad, fun, np.zeros(n), "lbfgs", 200, 10, gtol=1e-10)
    assert status == 0
    assert np.linalg.norm(x - xs) < 1e-6 * np.linalg.norm(xs)
    assert all(hist[i + 1] <= hist[i] for i in range(len(hist) - 1))


def test_assimilate_reduces_cost_and_metric_equivalence():
    N, steps = 16, 10
    ph = Physics(N=N, nu=1e-2, dt=1e-2)
    obs = _twin_obs(N, ph, steps, [0, 5, 10], 2, seed=21)
    fg = np.zeros((N, N))
    w1, h1, it1, st1 = O.assimilate(fg, ph, steps, obs, precond.Kernel(1, 0.1), "lbfgs", 4)
    assert st1 == 0 and h1[-1] < 0.5 * h1[0]
    # vorticity control == W = 1/k^2 velocity control (App. B): same iterates
    fg2 = O.init_field(N, [8], kind=0, k0=3.0)[0] * 0.5
    wa, ha, _, _ = O.assimilate(fg2, ph, steps, obs, precond.Kernel(2, 1.0, precond.VELOCITY), "lbfgs", 3)
    wb, hb, _, _ = O.assimilate(fg2, ph, steps, obs, precond.Kernel(0, 0.0, precond.VORTICITY), "lbfgs", 3)
    assert np.allclose(ha, hb, rtol=1e-10)
    assert np.linalg.norm(wa - wb) < 1e-9 * np.linalg.norm(wa)


# --------------------------------------------------------------- fields -----

def test_splitmix64_mix_is_a_bijection_and_uniform():
    # the finaliser is invertible (odd multipliers, xorshifts): undo it step by step
    def unxorshift(z, k):
        x = z.copy()
        for _ in range(64 // k + 1):
            x = z ^ (x >> np.uint64(k))
        return x
    inv1 = pow(0xBF58476D1CE4E5B9, -1, 1 << 64)
    inv2 = pow(0x94D049BB133111EB, -1, 1 << 64)
    idx = np.arange(1, 2001, dtype=np.uint64)
    z = fields.splitmix64(12345, idx)
    with np.errstate(over="ignore"):
        x = unxorshift(z, 31) * np.uint64(inv2)
        x = unxorshift(x, 27) * np.uint64(inv1)
        x = unxorshift(x, 30)
        state = np.uint64(12345) + idx * fields.GAMMA
    assert np.array_equal(x, state)
    u = fields.uniform01(fields.splitmix64(7, np.arange(1, 100001, dtype=np.uint64)))
    hist, _ = np.histogram(u, bins=20, range=(0, 1))
    chi2 = float(np.sum((hist - 5000.0) ** 2 / 5000.0))
    assert chi2 < 45.0                      # 19 dof, p ~ 1e-3
    assert u.min() >= 0.0 and u.max() < 1.0


def test_splitmix64_known_answers():
    """Known-answer pin of the generator: the published SplitMix64 stream seeded with 0 (the
    reference generator advances its state by the golden-ratio increment, then mixes it, so its
    n-th output is output n of this counter form).  A wrong increment or multiplier anywhere
    changes these."""
    z = fields.splitmix64(0, np.arange(1, 4, dtype=np.uint64))
    assert [int(v) for v in z] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    # uniforms are the top 53 bits
    assert fields.uniform01(z[:1])[0] == (0xE220A8397B1DCDAF >> 11) * 2.0 ** -53


@pytest.mark.parametrize("kind", [0, 1])
def test_init_field_energy_and_spectrum(kind):
    N = 64
    g = model.grid(N)
    w = O.init_field(N, [0, 1], kind=kind, k0=4.0, target=0.5)
    for b in range(2):
        u = g.apply(g.m_u, w[b])
        v = g.apply(g.m_v, w[b])
        assert abs(0.5 * np.mean(u * u + v * v) - 0.5) < 1e-14
        wh = dft.fft2(w[b])
        # real field with spectrum inside S only
        assert np.max(np.abs(wh * (1 - g.mask))) < 1e-10 * np.max(np.abs(wh))
        if kind == 0:
            # random phase: |w_hat|^2 / (k E(k)) is the same for every mode in S
            kap = np.sqrt(g.k2)
            Ek = fields.energy_spectrum(np.where(g.k2 > 0, kap, 1.0), 4.0)
            sel = (g.mask > 0) & (Ek > 1e-8 * Ek.max())
            ratio = np.abs(wh[sel]) ** 2 / (kap[sel] * fields.energy_spectrum(kap[sel], 4.0))
            assert np.max(ratio) / np.min(ratio) - 1 < 1e-9
    assert np.max(np.abs(w[0] - w[1])) > 0.1


def test_init_field_keyed_by_wavevector():
    # the same seed draws the same phases for the shared modes at two grid sizes
    a = O.init_field(32, [5], kind=2, target=1.0)[0]
    b = O.init_field(64, [5], kind=2, target=1.0)[0]
    ga, gb = model.grid(32), model.grid(64)
    ha, hb = dft.fft2(a), dft.fft2(b)
    for kx, ky in [(1, 0), (2, 3), (-4, 5), (7, -2)]:
        za = ha[ky % 32, kx % 32]
        zb = hb[ky % 64, kx % 64]
        assert abs(za / abs(za) - zb / abs(zb)) < 1e-12


def test_white_noise_rms():
    w = O.init_field(32, [3], kind=2, target=1e-2)[0]
    assert abs(np.sqrt(np.mean(w * w)) - 1e-2) < 1e-16


def test_first_guess_recovers_band_limited_field():
    # a field whose modes all lie below the probe Nyquist is recovered exactly
    N, s = 32, 4
    g = model.grid(N)
    X, Y = np.meshgrid(g.x, g.y)
    w = np.cos(2 * X + Y) + 0.5 * np.sin(X - 3 * Y)
    o = model.observe(g, g.mask * dft.fft2(w), s)
    fg = fields.first_guess(N, s, o)
    assert np.max(np.abs(fg - w)) < 1e-13


# -------------------------------------------------------------- ensemble -----

def test_shell_binning_matches_brute_force():
    N = 16
    g = model.grid(N)
    idx = ensemble.shell_index(g)
    for q in range(N):
        for p in range(N):
            kx = p if p < N // 2 else p - N
            ky = q if q < N // 2 else q - N
            r = math.sqrt(kx * kx + ky * ky)
            assert idx[q, p] == int(math.floor(r + 1e-12))


def test_shells_linear_diffusion_closed_form():
    # forward field identically zero: Nl' = 0, so lambda_n = E(h)^(H-n) lambda_H exactly
    N, steps, nu, mu, h = 32, 30, 1e-2, 0.1, 1e-2
    ph = Physics(N=N, nu=nu, dt=h, mu=mu)
    g = model.grid(N)
    rows, _ = ensemble.impulse_adjoint(np.zeros((N, N)), ph, steps, 16, 16, 10)
    e = np.zeros((N, N)); e[16, 16] = 1.0
    lam0 = np.conj(g.m_u) * dft.fft2(e)
    idx = ensemble.shell_index(g)
    for n in [0, 1, 17, 30]:
        decay = np.exp(-(nu * g.k2 + mu) * h) ** (2 * n)
        ref = [float(np.sum((0.5 * g.k2 * np.abs(lam0) ** 2 * decay / N ** 4)[idx == k]))
               for k in range(1, 11)]
        assert np.allclose(rows[n], ref, rtol=1e-13, atol=0)


def test_growth_rate_fit_exact_exponentials():
    dt = 2e-3
    tau = np.arange(600) * dt
    rates = np.array([-1.0, 0.5, 3.0])
    E = np.exp(np.outer(tau, rates)) * np.array([2.0, 1e-3, 7.0])
    got = ensemble.growth_rates(E, dt)
    assert np.allclose(got, rates, rtol=1e-10)


def test_total_adjoint_energy_parseval_against_physical_velocity():
    # 1/2 sum_k |k|^2 |lam_hat|^2 / N^4 equals the grid mean of 1/2 (u^2 + v^2) of the adjoint
    # velocity u = d_y lam, v = -d_x lam, formed in physical space by the inverse DFT
    N = 16
    g = model.grid(N)
    lam = g.mask * dft.fft2(np.random.default_rng(3).standard_normal((N, N)))
    u = dft.ifft2(1j * g.iky * lam).real
    v = dft.ifft2(-1j * g.ikx * lam).real
    assert ensemble.total_energy(g, lam) == pytest.approx(float(np.mean(0.5 * (u * u + v * v))), rel=1e-13)
    # every mode with |k| >= 1 lies in one shell: the shells partition the total
    nmax = int(math.isqrt(2 * (N // 2) ** 2)) + 1
    assert np.sum(ensemble.shell_energy(g, lam, nmax)) == pytest.approx(ensemble.total_energy(g, lam), rel=1e-13)


def test_ensemble_statistics_single_member_and_jensen():
    N, H = 16, 6
    ph = Physics(N=N, nu=1e-3, dt=5e-3)
    w = O.init_field(N, [1, 2, 3], kind=0, k0=3.0)
    one = ensemble.ensemble_statistics([w[0]], ph, H, 5, 9, 8)
    assert np.array_equal(one["energy_of_mean"], one["mean_energy"])
    assert np.allclose(one["snr"], 1.0, rtol=0, atol=1e-15)
    # identical members: the mean is the member
    two = ensemble.ensemble_statistics([w[0], w[0]], ph, H, 5, 9, 8)
    assert np.allclose(two["energy_of_mean"], one["energy_of_mean"], rtol=1e-14, atol=0)
    # different members: the energy of the mean never exceeds the mean energy (Jensen), per shell and total
    st = ensemble.ensemble_statistics(list(w), ph, H, 5, 9, 8)
    assert np.all(st["energy_of_mean"] <= st["mean_energy"] * (1 + 1e-12))
    assert np.all(st["snr"] <= 1 + 1e-12) and np.all(st["snr"] > 0)
    # at the terminal step every member holds the same impulse: the mean is that impulse
    assert st["snr"][0] == pytest.approx(1.0, rel=1e-14)
    assert np.all(st["snr"][1:] < 1)
    # mean energy is the average of the single-member rows
    rows = [ensemble.impulse_adjoint(x, ph, H, 5, 9, 8)[0] for x in w]
    assert np.allclose(st["mean_energy"], np.mean(rows, axis=0), rtol=1e-14, atol=0)


# ---------------------------------------------------- regularisation, metrics -----

def _grad_u_squared(g, w_hat):
    """int |grad u|^2 dOmega on the grid from the velocity of w_hat, its four
    derivatives formed spectrally (independent of the omega^2 form)."""
    u_hat = g.m_u * w_hat
    v_hat = g.m_v * w_hat
    tot = 0.0
    for f in (u_hat, v_hat):
        for d in (1j * g.ikx, 1j * g.iky):
            q = dft.ifft2(d * f).real
            tot += float(np.sum(q * q))
    return tot * (2 * np.pi / g.N) ** 2


def test_sobolev_term_equals_velocity_gradient_integral():
    N, lam = 32, 0.37
    g = model.grid(N)
    w_hat = g.mask * dft.fft2(O.init_field(N, [4], kind=0, k0=5.0)[0])
    assert model.sobolev_term(g, w_hat, lam) == pytest.approx(0.5 * lam * _grad_u_squared(g, w_hat), rel=1e-12)


def test_sobolev_gradient_finite_differences_and_zero_residual_closed_form():
    N, steps, lam = 16, 10, 2e-3
    ph = Physics(N=N, nu=1e-3, dt=5e-3)
    osteps = [0, 5, 10]
    obs = _twin_obs(N, ph, steps, osteps, 4, seed=21)
    w0 = O.init_field(N, [22], kind=0, k0=3.0)[0]
    J, grad = adjoint.adjoint_gradient(w0, ph, steps, obs, sobolev=lam)
    d = np.random.default_rng(5).standard_normal((N, N))
    eps = 1e-6
    Jp = model.forward(w0 + eps * d, ph, steps, obs, sobolev=lam)[1]
    Jm = model.forward(w0 - eps * d, ph, steps, obs, sobolev=lam)[1]
    assert (Jp - Jm) / (2 * eps) == pytest.approx(float(np.sum(grad * d)), rel=1e-6)
    # observations of the field itself: the residual vanishes, J and its gradient are the term alone
    g = model.grid(N)
    _, _, own = model.forward(w0, ph, steps, Obs(4, osteps))
    J0, g0 = adjoint.adjoint_gradient(w0, ph, steps, Obs(4, osteps, own), sobolev=lam)
    w_hat = g.mask * dft.fft2(w0)
    assert J0 == pytest.approx(0.5 * lam * _grad_u_squared(g, w_hat), rel=1e-12)
    # gradient of (lam/2) int omega^2 in the grid inner product: lam (2 pi/N)^2 P omega0
    Pw = g.to_phys(1.0, w_hat)
    assert np.allclose(g0, lam * (2 * np.pi / N) ** 2 * Pw, rtol=0, atol=1e-14 * np.abs(Pw).max())


def test_streamfunction_metric():
    N = 32
    g = model.grid(N)
    w = O.init_field(N, [9], kind=0, k0=5.0)[0]
    # W = |k|^2 (fractional, alpha = -1) in the velocity metric is the identity in the streamfunction metric
    a = precond.precondition(w, precond.Kernel(precond.FRACTIONAL, -1.0, precond.VELOCITY), -0.5)
    b = precond.precondition(w, precond.Kernel(precond.IDENTITY, 0.0, precond.STREAMFUNCTION), -0.5)
    assert np.allclose(a, b, rtol=0, atol=1e-12 * np.abs(b).max())
    # with W = 1 the latent control's Euclidean norm is the streamfunction's: psi_hat = omega_hat / |k|^2
    psi = dft.ifft2(g.mask * g.inv_k2 * dft.fft2(w)).real
    assert float(np.sum(b * b)) == pytest.approx(float(np.sum(psi * psi)), rel=1e-12)


# ----------------------------------------------------- checkpoint schedules

def _binom_beta(a, t):
    """beta(a, t) = C(a + t, a): steps reversible with a snapshots and t advances per step (0 for t < 0)."""
    return math.comb(a + t, a) if t >= 0 else 0


def test_checkpoint_cost_matches_binomial_closed_form():
    # Griewank & Walther: with the first state held and s free slots, let t be the
    # least integer with beta(s + 1, t) >= l; the fewest advances are t l - beta(s + 2, t - 1)
    for s in range(1, 7):
        for l in range(1, 90):
            t = 0
            while _binom_beta(s + 1, t) < l:
                t += 1
            assert O.min_advances(l, s) == t * l - _binom_beta(s + 2, t - 1), (l, s)


def test_checkpoint_cost_special_cases():
    for l in range(1, 40):
        assert O.min_advances(l, 0) == l * (l - 1) // 2       # no slot: every step from the start
        assert O.min_advances(l, max(l - 1, 0)) == l - 1      # a slot per step: each advanced once
        assert O.min_advances(l, l + 5) == l - 1
    # optimal first advances of the closed form's range
    for s in range(1, 6):
        for l in range(2, 60):
            t = 0
            while _binom_beta(s + 1, t) < l:
                t += 1
            lo = max(_binom_beta(s + 1, t - 2), l - _binom_beta(s, t), 1)
            hi = min(_binom_beta(s + 1, t - 1), l - _binom_beta(s, t - 1))
            assert O.optimal_first_advances(l, s) == list(range(lo, hi + 1)), (l, s)


def _exhaustive_min_advances(l, s):
    """Fewest unit advances over every strategy (not only recursive ones): states are
    (live position or -1, held snapshot positions, steps left to reverse).  Moves:
    advance the live state one step (cost 1), store it, drop a snapshot other than
    the first, restore a snapshot, or reverse the next step when the live state is
    at its start."""
    import collections
    start = (0, frozenset([0]), l)
    dist = {start: 0}
    dq = collections.deque([start])
    while dq:
        st = dq.popleft()
        live, snaps, r = st
        d = dist[st]
        if r == 0:
            return d
        moves = []
        if 0 <= live < r - 1:
            moves.append(((live + 1, snaps, r), 1))
        if live >= 0 and live not in snaps and len(snaps) < s + 1:
            moves.append(((live, snaps | {live}, r), 0))
        for q in snaps:
            if q != 0:
                moves.append(((live, snaps - {q}, r), 0))
            moves.append(((q, snaps, r), 0))
        if live == r - 1:
            moves.append(((-1, snaps, r - 1), 0))
        for nst, c in moves:
            if nst not in dist or dist[nst] > d + c:
                dist[nst] = d + c
                if c == 0:
                    dq.appendleft(nst)
                else:
                    dq.append(nst)
    raise AssertionError("unreachable")


def test_checkpoint_cost_is_the_optimum_over_all_strategies():
    for s in range(0, 4):
        for l in range(1, 9):
            assert O.min_advances(l, s) == _exhaustive_min_advances(l, s), (l, s)


# ------------------------------------------------- truth-field statistics

def _table2():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "truth_statistics_table2.txt")
    rows, re_l = {}, None
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        if f[0] == "HIT_Re_L":
            re_l = float(f[1])
            continue
        rows[f[0]] = dict(zip(("Re", "u_rms", "lambda", "Re_lambda", "Omega", "eps", "chi", "k_eta"),
                              map(float, f[1:])))
    return rows, re_l


def test_table2_printed_statistics_obey_their_definitions():
    # the paper's printed numbers satisfy the caption's definitions to their printed precision,
    # which fixes the reading of each quantity used by oracle.stats
    rows, re_l = _table2()
    for name, r in rows.items():
        nu = 1.0 / r["Re"]
        assert r["u_rms"] * r["lambda"] / nu == pytest.approx(r["Re_lambda"], rel=1e-2), name
        assert 2.0 * nu * r["Omega"] == pytest.approx(r["eps"], rel=1e-2), name       # eps = nu <|grad u|^2> = 2 nu Omega
        assert abs((r["chi"] / nu ** 3) ** (1.0 / 6.0) - r["k_eta"]) <= 0.5, name   # printed to integers
        # Taylor microscale of an isotropic field, lambda = u_rms / rms(du/dx) = u_rms sqrt(2 / Omega)
        assert r["u_rms"] * math.sqrt(2.0 / r["Omega"]) == pytest.approx(r["lambda"], rel=3e-2), name
    hit = rows["HIT"]
    assert hit["u_rms"] * 2.0 * math.pi * hit["Re"] == pytest.approx(re_l, rel=1e-2)


def test_turbulence_statistics_single_mode_and_identities():
    from oracle.stats import turbulence_statistics
    N, k, nu = 32, 3, 2e-3
    x = 2 * np.pi * np.arange(N) / N
    w = np.tile(np.cos(k * x), (N, 1))          # omega = cos(k x): v = sin(k x) / k, u = 0
    st = turbulence_statistics(w, nu)
    assert st["Omega"] == pytest.approx(0.25, rel=1e-13)
    assert st["u_rms"] == pytest.approx(1.0 / (2 * k), rel=1e-13)
    assert st["eps"] == pytest.approx(nu / 2, rel=1e-13)
    assert st["chi"] == pytest.approx(nu * k * k / 2, rel=1e-13)
    assert st["k_eta"] == pytest.approx((k * k / (2 * nu * nu)) ** (1.0 / 6.0), rel=1e-13)
    # on a turbulent field: eps = 2 nu Omega (periodic, divergence-free) and u_rms^2 = the energy
    w = O.init_field(N, [5], kind=0, k0=4.0, target=0.5)[0]
    st = turbulence_statistics(w, nu)
    assert st["eps"] == pytest.approx(2 * nu * st["Omega"], rel=1e-12)
    assert st["u_rms"] ** 2 == pytest.approx(0.5, rel=1e-12)
    assert st["Re_lambda"] == pytest.approx(st["u_rms"] * st["lambda"] / nu, rel=1e-14)


def test_stored_oracle_fixtures_are_intact():
    # the full-horizon expectations written by tests/golden/make_oracle_fixtures.py: shapes, and the parts
    # that are cheap to recompute (the step-0 observations of the c1 truth; the terminal impulse row)
    import os
    gold = os.path.join(os.path.dirname(__file__), "golden")
    c1 = np.load(os.path.join(gold, "c1_full_horizon.npz"))
    assert c1["obs"].shape == (5, 2, 32, 32) and c1["grad"].shape == (256, 256)
    assert list(c1["obs_steps"]) == [0, 250, 500, 750, 1000]
    assert np.all(np.isfinite(c1["grad"])) and float(c1["J"]) > 0
    truth = O.init_field(256, [0], kind=0, k0=10.0, target=0.5)[0]
    ph = Physics(N=256, nu=1e-4, dt=2e-3)
    obs0 = O.forward(truth, ph, 0, Obs(8, [0]))[2][0]
    assert np.allclose(c1["obs"][0], obs0, rtol=0, atol=1e-13 * np.abs(obs0).max())
    sh = np.load(os.path.join(gold, "ensemble_member17.npz"))["shells"]
    assert sh.shape == (501, 85) and np.all(np.isfinite(sh))
    g = model.grid(256)
    e = np.zeros((256, 256))
    e[128, 128] = 1.0
    row0 = ensemble.shell_energy(g, np.conj(g.m_u) * dft.fft2(e), 85)
    assert np.allclose(sh[0], row0, rtol=1e-13, atol=0)
    c2 = np.load(os.path.join(gold, "c2_100_steps.npz"))
    assert c2["obs"].shape == (3, 2, 32, 32) and c2["grad"].shape == (512, 512) and c2["omega_T"].shape == (512, 512)
    assert list(c2["obs_steps"]) == [0, 50, 100]
    assert np.all(np.isfinite(c2["grad"])) and np.all(np.isfinite(c2["omega_T"])) and float(c2["J"]) > 0
    ph2 = Physics(N=512, nu=1.0 / 40, dt=1e-3, mu=0.1, forcing_amp=1.0, forcing_k=4)
    truth2 = O.init_field(512, [1], kind=0, k0=6.0, target=0.5)[0]
    obs20 = O.forward(truth2, ph2, 0, Obs(16, [0]))[2][0]
    assert np.allclose(c2["obs"][0], obs20, rtol=0, atol=1e-13 * np.abs(obs20).max())
    # the L-BFGS fixtures: shapes, the step-0 probes and the interpolated first guess recomputed,
    # cost histories finite, decreasing and sharing their prefixes (a longer run repeats a shorter one)
    for name, N, stride, seed, k0, ph_f, iters in (
            ("c1_grid_lbfgs.npz", 256, 8, 0, 10.0, ph, (1, 5, 10)),
            ("c2_grid_lbfgs.npz", 512, 16, 1, 6.0, ph2, (1, 3, 5))):
        lb = np.load(os.path.join(gold, name))
        M = N // stride
        assert lb["obs"].shape[1:] == (2, M, M) and lb["first_guess"].shape == (N, N)
        tr = O.init_field(N, [seed], kind=0, k0=k0, target=0.5)[0]
        o0 = O.forward(tr, ph_f, 0, Obs(stride, [0]))[2][0]
        assert np.allclose(lb["obs"][0], o0, rtol=0, atol=1e-13 * np.abs(o0).max())
        assert np.allclose(lb["first_guess"], O.first_guess(N, stride, lb["obs"][0]), rtol=0, atol=1e-13)
        hists = [lb[f"J_hist_{k}"] for k in iters]
        ev = int(lb["sample_every"]) if "sample_every" in lb else 1
        for k, h in zip(iters, hists):
            assert h.shape == (k + 1,) and np.all(np.isfinite(h)) and np.all(np.diff(h) < 0)
            assert lb[f"omega_{k}"].shape == (N // ev, N // ev) and np.all(np.isfinite(lb[f"omega_{k}"]))
        for a, b in zip(hists, hists[1:]):   # equal up to the BLAS's summation order
            assert np.allclose(a, b[:len(a)], rtol=1e-12, atol=0)
    g1k = np.load(os.path.join(gold, "grid1024_50_steps.npz"))
    ev = int(g1k["sample_every"])
    assert g1k["omega_T"].shape == (1024 // ev, 1024 // ev) and g1k["grad"].shape == (1024 // ev, 1024 // ev)
    assert list(g1k["obs_steps"]) == [0, 25, 50] and g1k["obs"].shape == (3, 2, 64, 64)
    assert np.all(np.isfinite(g1k["grad"])) and float(g1k["J"]) > 0
