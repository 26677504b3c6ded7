"""GPU RPCA ADMM driver (Appendix B) against the oracle driver: identical
start, the same number of iterations, each side with its own power-iteration
bound.  Per-iteration quantities agree to FP32 rounding; the drift after a few
iterations is bounded (ADMM is non-expansive)."""
import numpy as np
import pytest

import synth
from oracle import drivers, metrics

pytestmark = pytest.mark.gpu


def _admm_pair(m, n, iters, K, inv_rho, eta_over_rho, seed):
    import torch
    import paper_1705_07112_amd as cpa
    I, _, _ = synth.rpca_frames(m, n, rank=min(40, m // 4), outlier_frac=0.05, seed=seed)
    Id = torch.from_numpy(I).cuda()
    opts = cpa.Opts(K=K, warm_start=True, power_iters=100)
    run = cpa.RpcaAdmm(Id, inv_rho, eta_over_rho, opts)
    Et = torch.zeros(iters, dtype=torch.float64, device="cuda")
    run.iterate(iters, Et)
    torch.cuda.synchronize()
    l_o, s_o, E_o, _ = drivers.rpca_admm(I.astype(np.float64), inv_rho, eta_over_rho, iters, K)
    return run.L.cpu().numpy(), run.S.cpu().numpy(), Et.cpu().numpy(), l_o, s_o, np.array(E_o)


def test_admm_small_matches_oracle():
    print("admm 96x80 12 iterations", flush=True)
    l, s, E, l_o, s_o, E_o = _admm_pair(96, 80, 12, 20, 1.0, 1.0 / np.sqrt(96), 11)
    el, es = metrics.rel_fro(l, l_o), metrics.rel_fro(s, s_o)
    print(f"  l {el:.3e} s {es:.3e} E {E[:4]} vs {E_o[:4]}", flush=True)
    assert el < 1e-4 and es < 1e-3
    assert np.max(np.abs(E - E_o) / np.maximum(E_o, 1e-12)) < 1e-3


def test_admm_full_size_first_iterations():
    """The bench workload (1024 x 1024, K = 30, 1/rho = 10, eta = 1/32) for 3 iterations."""
    print("admm 1024x1024 3 iterations", flush=True)
    l, s, E, l_o, s_o, E_o = _admm_pair(1024, 1024, 3, 30, 10.0, 10.0 / 32.0, synth.BASE_SEED + 1)
    el, es = metrics.rel_fro(l, l_o), metrics.rel_fro(s, s_o)
    print(f"  l {el:.3e} s {es:.3e} E {E} vs {E_o}", flush=True)
    assert el < 1e-5 and es < 1e-4
    assert np.max(np.abs(E - E_o) / np.maximum(E_o, 1e-12)) < 1e-4
