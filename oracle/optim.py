"""Steepest descent and L-BFGS in the latent control (oracle).

Test infrastructure only (see ``oracle/__init__.py``).

The paper runs L-BFGS (Nocedal 1980; Liu & Nocedal 1989) in the Euclidean
metric on the latent control s0 = G^{-1/2} u0 and maps back with G^{1/2} after
each update (Sec. II.C).  It gives no memory size, initial Hessian, line
search or stopping rule; this oracle uses the textbook choices:

* two-loop recursion with m stored pairs and H0 = gamma I,
  gamma = s^T y / y^T y of the newest pair;
* first iteration, or a search direction that is not a descent direction:
  d = -g with trial step J / |g|^2 (Polyak step toward J = 0) and the memory
  cleared; otherwise trial step 1;
* backtracking Armijo rule J(s + a d) <= J(s) + 1e-4 a g^T d, halving a at
  most 30 times; failure stops the run (the paper's "step size collapses",
  Sec. III.C-D);
* a pair (s_k, y_k) is stored only if s_k^T y_k > 1e-10 |s_k| |y_k|.

Steepest descent uses d = -g with the same trial step and Armijo rule.
"""

import numpy as np

from .adjoint import adjoint_gradient
from .model import forward
from .precond import precondition

ARMIJO_C1 = 1e-4
MAX_TRIALS = 30
CURV_EPS = 1e-10


def lbfgs_two_loop(g, pairs):
    """Return H g for the L-BFGS inverse-Hessian built from pairs [(s, y), ...] (oldest first)."""
    q = g.copy()
    alphas = []
    rhos = [1.0 / float(np.dot(y, s)) for (s, y) in pairs]
    for (s, y), rho in zip(reversed(pairs), reversed(rhos)):
        a = rho * float(np.dot(s, q))
        alphas.append(a)
        q = q - a * y
    s_new, y_new = pairs[-1]
    gamma = float(np.dot(s_new, y_new)) / float(np.dot(y_new, y_new))
    r = gamma * q
    for (s, y), rho, a in zip(pairs, rhos, reversed(alphas)):
        b = rho * float(np.dot(y, r))
        r = r + (a - b) * s
    return r


def minimize(fun_grad, fun, x0, method="lbfgs", max_iter=10, m=10, gtol=0.0):
    """Generic driver on flat vectors.

    fun_grad(x) -> (J, g); fun(x) -> J.  Returns (x, J history, iterations
    completed, status) with status 0 = ok, -5 = line-search failure.  The
    gradient is evaluated at the iterates that start an iteration only (the
    last accepted point needs J alone).  With gtol > 0 the run also stops
    (status 0) once |g| <= gtol.
    """
    x = np.array(x0, dtype=np.float64)
    J, g = fun_grad(x)
    hist = [J]
    pairs = []
    status = 0
    done = 0
    for it in range(max_iter):
        if gtol > 0.0 and float(np.linalg.norm(g)) <= gtol:
            break
        use_memory = method == "lbfgs" and len(pairs) > 0
        if use_memory:
            d = -lbfgs_two_loop(g, pairs)
            gd = float(np.dot(g, d))
            if gd >= 0.0:
                pairs = []
                use_memory = False
        if use_memory:
            alpha = 1.0
        else:
            d = -g
            gd = float(np.dot(g, d))
            alpha = J / float(np.dot(g, g))
        accepted = False
        for _trial in range(MAX_TRIALS):
            x_try = x + alpha * d
            J_try = fun(x_try)
            if J_try <= J + ARMIJO_C1 * alpha * gd:
                accepted = True
                break
            alpha *= 0.5
        if not accepted:
            status = -5
            break
        done = it + 1
        if it == max_iter - 1:
            x, J = x_try, J_try
            hist.append(J)
            break
        J_new, g_new = fun_grad(x_try)
        if method == "lbfgs":
            sk = x_try - x
            yk = g_new - g
            sy = float(np.dot(sk, yk))
            if sy > CURV_EPS * np.linalg.norm(sk) * np.linalg.norm(yk):
                pairs.append((sk, yk))
                if len(pairs) > m:
                    pairs.pop(0)
        x, g, J = x_try, g_new, J_new
        hist.append(J)
    return x, hist, done, status


def assimilate(omega_fg, phys, n_steps, obs, kern, method="lbfgs", max_iter=10, m=10, sobolev=0.0):
    """Preconditioned 4D-Var from a first guess (Sec. II.C).

    Optimises the latent s = precondition(omega, -1/2); every evaluation maps
    back with omega0 = precondition(s, +1/2) and the latent gradient is
    precondition(dJ/d omega0, +1/2).  sobolev = lambda > 0 adds the
    regularisation term of Eq. (4) to the cost.  Returns (omega0 estimate,
    J history, iterations, status).
    """
    N = phys.N
    shape = (N, N)

    def to_phys(x):
        return precondition(x.reshape(shape), kern, 0.5)

    def fun_grad(x):
        J, g = adjoint_gradient(to_phys(x), phys, n_steps, obs, sobolev)
        return J, precondition(g, kern, 0.5).ravel()

    def fun(x):
        _w, J, _o = forward(to_phys(x), phys, n_steps, obs, sobolev)
        return J

    s0 = precondition(np.asarray(omega_fg, dtype=np.float64), kern, -0.5).ravel()
    x, hist, it, status = minimize(fun_grad, fun, s0, method, max_iter, m)
    return to_phys(x), hist, it, status
