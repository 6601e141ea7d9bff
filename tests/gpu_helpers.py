"""Shared helpers of the GPU parity tests: move populations between the
oracle's [P, d] layout and the HIP path's [d, P] layout."""
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
