"""Implicit Euler time stepping around the solvers (FP64).

One step (Background, Optimization-Based Integration, and its footnote):
  1. x~ = x^t + h v^t;
  2. Dirichlet vertices are set to their step targets, giving the predictor
     x^_0 (this package's reading: targets are imposed on the predictor);
  3. the iteration starts from x^_0, or from a proposal x_p when
     E(x_p) < E(x^_0) (the acceptance rule of the learned warm start); with
     several proposals, each in turn replaces the start when its E is below
     the current start's, so the start has the least E among them and x^_0;
  4. x^{t+1} = argmin E by the chosen solver;
  5. v^{t+1} = (x^{t+1} - x^t) / h for every vertex (Dirichlet vertices get
     their kinematic velocity).
Quasistatic problems skip the inertia term and start from the previous
solution with updated targets.

Pins: tests/test_oracle_timestep.py -- momentum balance of a free body,
a body at rest without gravity stays at rest.
"""
import numpy as np

from .solvers import newton, solve


def predictor(prob, x_t, v_t, targets):
    if prob.quasistatic:
        xh = np.array(x_t, dtype=np.float64, copy=True)
    else:
        xh = x_t + prob.h * v_t
    prob.set_inertial_target(xh if not prob.quasistatic else prob.X)
    fx = prob.fixed
    xh = xh.copy()
    xh[fx] = targets[fx]
    return xh


def step(prob, x_t, v_t, targets, basis, params, tol, colours=None, proposal=None,
         record=False):
    """One implicit step; returns (x, v, SolveResult, accepted): accepted is
    0, or k when the k-th proposal (1-based; `proposal` one array or a list)
    is the start."""
    xh = predictor(prob, x_t, v_t, targets)
    x0 = xh
    accepted = 0
    if proposal is not None:
        props = proposal if isinstance(proposal, (list, tuple)) else [proposal]
        E0 = prob.energy(xh)
        for k, pr in enumerate(props):
            xp = np.array(pr, dtype=np.float64, copy=True)
            xp[prob.fixed] = xh[prob.fixed]
            Ep = prob.energy(xp)
            if Ep < E0:
                x0, E0, accepted = xp, Ep, k + 1
    res = solve(prob, x0, basis, params, tol, colours=colours, x_hat0=xh, record=record)
    v = (res.x - x_t) / prob.h if not prob.quasistatic else np.zeros_like(x_t)
    return res.x, v, res, accepted


def newton_step(prob, x_t, v_t, targets, tol=1e-10, record=False):
    xh = predictor(prob, x_t, v_t, targets)
    res = newton(prob, xh, tol=tol, x_hat0=xh, record=record)
    v = (res.x - x_t) / prob.h if not prob.quasistatic else np.zeros_like(x_t)
    return res.x, v, res
