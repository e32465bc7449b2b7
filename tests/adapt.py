"""Converts the seeded workload specs into the oracle's own problem description."""
import oracle as O
from paper_1108_1688_amd import workloads as W


def to_oracle(s: W.SolveSpec) -> O.Problem:
    axes = [O.Axis(a.n, a.z_min, a.z_max, a.center, a.alpha, a.lo_face, a.hi_face) for a in s.axes]
    m = s.model
    return O.Problem(axes, kappa=m.kappa, theta_v=m.theta_v, lam=m.lam, gamma=m.gamma,
                     epsilon=m.epsilon, rho=m.rho, f_level=m.f_level, f_slope=m.f_slope,
                     f_decay=m.f_decay, kind=s.payoff.kind, expiry=s.payoff.expiry,
                     pay=s.payoff.pay, strike=s.payoff.strike, n_steps=s.n_steps,
                     scheme=s.scheme, theta=s.theta, soften=s.payoff.soften,
                     af_iters=s.af_iters, curve_t=m.curve_t, curve_p=m.curve_p)
