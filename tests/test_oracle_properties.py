"""Property-based pins of the CPU oracle (hypothesis): identities that hold for
every admissible input, checked on randomly drawn small problems rather than
on a few fixed seeds.

* The discrete adjoint is the exact transpose of the tangent-linear model
  (Sec. II.A, Eqs. (11)-(12); Sec. III: summation by parts to machine
  precision): <M' d, m> = <d, M'^T m> for random physics, horizons, base
  fields and directions.
* The preconditioner maps are inverse to each other on the de-aliased band
  (Sec. II.B-C, Eqs. (18)-(19)): precondition(precondition(f, -1/2), +1/2)
  is the band projection of f, for every kernel family and metric.
* The cost gradient matches a central difference of the cost (Eq. (12)).
"""

import numpy as np
from hypothesis import given, settings, strategies as st

import oracle as O
from oracle import model, precond
from oracle.model import Obs, Physics

SETTINGS = settings(max_examples=20, deadline=None, derandomize=True)

physics = st.builds(
    lambda N, nu, mu, amp, dt: Physics(N=N, nu=nu, dt=dt, mu=mu, forcing_amp=amp, forcing_k=2),
    N=st.sampled_from([8, 16]),
    nu=st.floats(0.0, 2e-2),
    mu=st.floats(0.0, 0.2),
    amp=st.floats(0.0, 1.0),
    dt=st.floats(1e-3, 1e-2),
)


@SETTINGS
@given(ph=physics, steps=st.integers(1, 6), seed=st.integers(0, 2 ** 31 - 1))
def test_adjoint_is_the_transpose_of_the_tangent(ph, steps, seed):
    rng = np.random.default_rng(seed)
    N = ph.N
    w0 = O.init_field(N, [seed % 1000], kind=0, k0=2.0)[0]
    d = rng.standard_normal((N, N))
    m = rng.standard_normal((N, N))
    lhs = float(np.sum(O.tlm_trajectory(w0, d, ph, steps) * m))
    rhs = float(np.sum(d * O.adjoint.adjoint_trajectory(w0, m, ph, steps)))
    scale = np.linalg.norm(O.tlm_trajectory(w0, d, ph, steps)) * np.linalg.norm(m)
    assert abs(lhs - rhs) <= 1e-13 * scale


kernels = st.one_of(
    st.builds(lambda m: precond.Kernel(0, 0.0, m), st.integers(0, 2)),
    st.builds(lambda s, m: precond.Kernel(1, s, m), st.floats(0.0, 0.5), st.integers(0, 2)),
    st.builds(lambda b, m: precond.Kernel(2, b, m), st.floats(-1.0, 1.0), st.integers(0, 2)),
    st.builds(lambda c, m: precond.Kernel(3, c, m), st.floats(0.0, 0.02), st.integers(0, 2)),
)


@SETTINGS
@given(kern=kernels, N=st.sampled_from([8, 16]), seed=st.integers(0, 2 ** 31 - 1))
def test_latent_maps_are_inverse_on_the_band(kern, N, seed):
    rng = np.random.default_rng(seed)
    f = rng.standard_normal((N, N))
    g = model.grid(N)
    band = g.apply(g.mask, f)                  # P f: the de-aliased band without the mean
    back = O.precondition(O.precondition(f, kern, -0.5), kern, 0.5)
    assert np.linalg.norm(back - band) <= 1e-12 * np.linalg.norm(band)


@SETTINGS
@given(ph=physics, steps=st.integers(1, 5), seed=st.integers(0, 2 ** 31 - 1))
def test_cost_gradient_matches_a_central_difference(ph, steps, seed):
    rng = np.random.default_rng(seed)
    N = ph.N
    truth = O.init_field(N, [seed % 997], kind=0, k0=2.0)[0]
    osteps = sorted({0, steps})
    _, _, mo = O.forward(truth, ph, steps, Obs(4, osteps))
    obs = Obs(4, osteps, mo)
    w0 = O.init_field(N, [(seed + 1) % 997], kind=0, k0=2.0)[0]
    J, grad = O.adjoint_gradient(w0, ph, steps, obs)
    d = rng.standard_normal((N, N))
    eps = 1e-5
    Jp = O.forward(w0 + eps * d, ph, steps, obs)[1]
    Jm = O.forward(w0 - eps * d, ph, steps, obs)[1]
    fd = (Jp - Jm) / (2 * eps)
    an = float(np.sum(grad * d))
    assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-8 * J) + 1e-10
