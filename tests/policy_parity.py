"""End-to-end policy parity of a march against the oracle (eq. nonlinear_sys with the tie rule of the search).

A step's policy is a unique correct result only at nodes where the oracle's decision at its own converged
step is clear: a single control within tau of the minimum (ties == 1) and every other control more than
1e3 * tau above it (margin).  There the GPU policy must equal the oracle's index for index.  Elsewhere several
policies are correct results (certified near-ties): those nodes are counted and their values are covered by
the value bound.  Each step of the GPU march is also checked on its own terms: the oracle's search started
from the GPU policy at the GPU's values changes nothing (the GPU policy is the tie rule's fixed point), and
the residual of the discrete HJB system at the GPU's values, max_k (A^k X - F^k) = X - U - dt min_k G_k,
is below the value bound (its infinity norm bounds |X - X*|_inf for these M-matrices, Section 3.4).
"""
import numpy as np

import oracle

MARGIN_FACTOR = 1e3


def _f_mid(pb, inst, t_prev, dt, theta):
    return pb.f_at(inst.f0, inst.f1, t_prev + theta * dt)


def check_march_policies(inst, ref, pol_gpu, vals_gpu=None, s=None, rel_tol=1e-10, log=None):
    """ref: oracle.march(inst, keep_policies=True, keep_values=True); pol_gpu: [n_steps][N] int16;
    vals_gpu (optional): [n_steps+1][N] FP64, U^0 .. U^N of the GPU march.  Returns the near-tie count."""
    pb = oracle.Problem(inst, s=s)
    I = pb.interior
    times = np.concatenate([[0.0], np.cumsum(inst.dts)])
    near_total = 0
    sure_total = 0
    for n in range(len(inst.dts)):
        dt, th = float(inst.dts[n]), float(inst.thetas[n])
        f = _f_mid(pb, inst, float(times[n]), dt, th)
        U0, X = ref["values"][n], ref["values"][n + 1]
        Xs = U0 if th == 0.0 else X       # an explicit step searches at U^{n-1}
        tau = pb.tau(Xs, U0, f)
        r = pb.improve(Xs, U0, th, f, tau, ref["policies"][n], want_extra=True)
        assert r["changed"] == 0, f"step {n}: the oracle's policy is not its own fixed point"
        sure = np.zeros(pb.N, bool)
        sure[I] = (r["ties"][I] == 1) & (r["margin"][I] >= MARGIN_FACTOR * tau)
        bad = np.nonzero(sure & (pol_gpu[n] != ref["policies"][n]))[0]
        assert bad.size == 0, (f"step {n}: {bad.size} policy mismatches at clear decisions, first node {bad[0]} "
                               f"gpu {pol_gpu[n][bad[0]]} oracle {ref['policies'][n][bad[0]]} "
                               f"margin/tau {r['margin'][bad[0]] / tau:.3g}")
        np.testing.assert_array_equal(pol_gpu[n][pb.bd], -1)
        near_total += int(I.size - np.count_nonzero(sure))
        sure_total += int(np.count_nonzero(sure))
        if vals_gpu is not None:
            Ug0, Xg = vals_gpu[n], vals_gpu[n + 1]
            Xgs = Ug0 if th == 0.0 else Xg
            taug = pb.tau(Xgs, Ug0, f)
            rg = pb.improve(Xgs, Ug0, th, f, taug, pol_gpu[n], want_extra=False)
            assert rg["changed"] == 0, f"step {n}: the GPU policy is not the tie rule's fixed point at its values"
            if th > 0.0:
                R = Xg[I] - Ug0[I] - dt * rg["gmin"][I]
                xinf = max(1.0, float(np.max(np.abs(Xg))))
                cmax = float(np.max(pb.c_of(pol_gpu[n]))) if inst.c is not None else 0.0
                bound = float(np.max(np.abs(R))) / (1.0 - th * dt * max(cmax, 0.0))
                assert bound <= rel_tol * xinf, f"step {n}: discrete HJB residual bound {bound:.3e}"
    if log is not None:
        log(f"  policies: {sure_total} clear decisions identical, {near_total} near-tie node-steps")
    return near_total
