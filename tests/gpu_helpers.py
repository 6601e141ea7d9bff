"""Shared helpers of the GPU parity tests: move populations between the
oracle's [P, d] layout and the HIP path's [d, P] layout."""
import math

import numpy as np
import torch

import oracle as O
import paper_1304_4334_amd as S


def gpu_model(w, precision=S.SMC_FP64, T=None):
    if T is not None and T != w.T:
        y = w.y[:T]
        X = None if w.X is None else w.X[:T]
        return S.Model(w.kind, y, X=X, K=w.K, shock=w.shock, precision=precision, I=w.I)
    return S.Model.from_workload(w, precision=precision)


def ora_model(w, T=None):
    return O.Model.from_workload(w, T=T)


def pop_to_gpu(gm, opop, max_chunk=64, with_grad=False):
    g = S.Population(gm, opop.J, opop.N, max_chunk=max_chunk, with_grad=with_grad)
    g.theta.copy_(torch.from_numpy(np.ascontiguousarray(opop.theta.T)))
    g.logprior.copy_(torch.from_numpy(opop.logprior))
    g.loglik.copy_(torch.from_numpy(opop.loglik))
    g.logw.copy_(torch.from_numpy(opop.logw))
    if gm.S > 0:
        g.state.copy_(torch.from_numpy(np.ascontiguousarray(opop.state[:, :gm.S].T)).to(g.state.dtype))
    return g


def theta_np(g):
    return g.theta.cpu().numpy().T.copy()


def sync():
    torch.cuda.synchronize()


def _log_u(seed, run, p, cycle, it):
    """log of the accept uniform of particle p: the first Philox word of
    counter (p, cycle, iteration, ACCEPT), ((x >> 11) + 1/2) 2^-53."""
    x = O.philox([int(p), int(cycle), int(it), O.ACCEPT], [int(seed), int(run)])[0]
    return math.log(((x >> 11) + 0.5) * 2.0 ** -53)


def accept_audit(gm, om, th, lp, ll, t, hl, seed, run, cycle, it, acc_g, acc_o, pidx=None,
                 kernel=S.SMC_KERNEL_RW, mean=None, g0_gpu=None):
    """Audit of Metropolis decisions taken with an FP32 likelihood recursion.

    For every particle (rows of th, global Philox indices pidx) the oracle's
    proposal and acceptance log-ratio Delta_o are rebuilt in FP64 from its
    definitions (Philox normals, hL, the oracle's densities), and the GPU's
    Delta_g from the same proposal evaluated by the GPU's own recursion
    (smc_loglik, and for the Langevin kernel the GPU's gradients).  Checks:
    the rebuilt oracle rule reproduces the oracle's decisions; the GPU took
    log u < Delta_g on every particle not within rounding of a tie; and every
    decision on which the two sides differ has log u between Delta_o and
    Delta_g (the flip is explained by the FP32 error of Delta alone).
    Returns (max |Delta_g - Delta_o| over finite values, number of flips)."""
    P, d = th.shape
    pidx = np.arange(P) if pidx is None else np.asarray(pidx)
    z = np.array([O.normals(seed, run, int(p), cycle, it, O.PROPOSAL, d) for p in pidx])
    logu = np.array([_log_u(seed, run, p, cycle, it) for p in pidx])

    def propose(g0):
        if kernel == S.SMC_KERNEL_INDEPENDENT:
            return mean[None, :] + z @ hl.T
        prop = th + z @ hl.T
        if kernel == S.SMC_KERNEL_MALA:
            prop = prop + 0.5 * (g0 @ hl) @ hl.T
        return prop

    def q_ratio(prop, g1):
        if kernel == S.SMC_KERNEL_RW:
            return np.zeros(P)
        if kernel == S.SMC_KERNEL_INDEPENDENT:
            wv = np.linalg.solve(hl, (th - mean[None, :]).T).T
        else:
            a = th - prop - 0.5 * (g1 @ hl) @ hl.T
            wv = np.linalg.solve(hl, a.T).T
        return -0.5 * (wv * wv).sum(1) + 0.5 * (z * z).sum(1)

    # oracle side, FP64
    g0_o = None
    if kernel == S.SMC_KERNEL_MALA:
        g0_o = np.array([O.loglik_grad(om, th[i], t)[1] + O.logprior_grad(om, th[i])[1]
                         for i in range(P)])
    prop_o = propose(g0_o)
    lp_o = np.array([O.logprior(om, prop_o[i]) for i in range(P)])
    ll_o = np.full(P, -np.inf)
    g1_o = np.zeros((P, d))
    for i in range(P):
        if lp_o[i] > -np.inf:
            if kernel == S.SMC_KERNEL_MALA:
                ll_o[i], g1_o[i] = O.loglik_grad(om, prop_o[i], t)
                g1_o[i] += O.logprior_grad(om, prop_o[i])[1]
            else:
                ll_o[i] = O.loglik(om, prop_o[i], t)[0]
    dlt_o = (lp_o + ll_o) - (lp + ll) + q_ratio(prop_o, g1_o)
    # GPU side: the same rule on the GPU's own densities (and gradients)
    prop_g = propose(g0_gpu) if kernel == S.SMC_KERNEL_MALA else prop_o
    lp_g = np.array([O.logprior(om, prop_g[i]) for i in range(P)])
    tg = torch.from_numpy(np.ascontiguousarray(prop_g.T)).cuda()
    ll_g = S.smc_loglik(gm, tg, t).cpu().numpy()
    ll_g = np.where(lp_g > -np.inf, ll_g, -np.inf)
    g1_g = np.zeros((P, d))
    if kernel == S.SMC_KERNEL_MALA:
        dl = torch.ones(P, dtype=torch.float64, device="cuda")
        g1_g = S.smc_loglik_backward(gm, tg, t, dl).cpu().numpy().T
        g1_g = g1_g + np.array([O.logprior_grad(om, prop_g[i])[1] for i in range(P)])
    dlt_g = (lp_g + ll_g) - (lp + ll) + q_ratio(prop_g, g1_g)
    with np.errstate(invalid="ignore"):
        dlt_o = np.where(np.isnan(dlt_o), -np.inf, dlt_o)
        dlt_g = np.where(np.isnan(dlt_g), -np.inf, dlt_g)
        # the rebuilt oracle rule is the oracle's
        tie_o = np.abs(logu - dlt_o) < 1e-9 * (1.0 + np.abs(dlt_o))
        assert np.array_equal((logu < dlt_o)[~tie_o], np.asarray(acc_o, bool)[~tie_o])
        # The GPU followed the rule on its own densities.  smc_loglik runs the
        # mutation kernel's recursion, but the two are compiled apart, so
        # their FP32 block sums may round differently: a decision within
        # 1e-6 of the likelihoods' size of a tie is not judged.  (The
        # Langevin kernel takes its value from the adjoint's forward sweep,
        # whose sums are grouped by segment: there the margin is 1e-4.)
        scale = 1.0 + np.abs(np.where(np.isfinite(ll_g), ll_g, 0.0)) + np.abs(ll)
        rel = 1e-4 if kernel == S.SMC_KERNEL_MALA else 1e-6
        tie_g = np.abs(logu - dlt_g) < rel * scale
        acc_g = np.asarray(acc_g, bool)
        bad = (acc_g != (logu < dlt_g)) & ~tie_g
        assert not bad.any(), (np.nonzero(bad)[0][:8], logu[bad][:4], dlt_g[bad][:4])
        # every flip lies between the two log-ratios (to the same margin)
        flip = acc_g != np.asarray(acc_o, bool)
        err = np.abs(dlt_g - dlt_o)
        ok = np.abs(logu - dlt_o) <= np.where(np.isfinite(err), err, np.inf) + rel * scale
        assert np.all(ok[flip]), (np.nonzero(flip & ~ok)[0][:8])
        fin = np.isfinite(dlt_o) & np.isfinite(dlt_g)
    max_err = float(err[fin].max()) if fin.any() else 0.0
    print(f"[audit] {P} decisions, {int(flip.sum())} flips, max |Delta_fp32 - Delta_fp64| "
          f"{max_err:.3e}, accepted {int(acc_g.sum())}")
    return max_err, int(flip.sum())
