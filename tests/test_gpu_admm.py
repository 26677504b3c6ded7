"""GPU RPCA ADMM driver (Appendix B) against the oracle driver.

Gated: one iteration started from the same state on both sides (the GPU's
own state, copied to the host) must agree to the FP32 tolerance -- the shrink
output z1 and the updated l, s, u.  Reported with a loose sanity bound: the
end-to-end drift after several iterations, where FP32 rounding is amplified
through the iteration."""
import numpy as np
import pytest

import synth
from oracle import drivers, metrics

pytestmark = pytest.mark.gpu

NAMES = ("l", "s", "z1", "z2", "u1", "u2", "u3")


def _state_host(run):
    return {k: run.block(i).cpu().numpy().astype(np.float64) for i, k in enumerate(NAMES)}


def _check_one_iteration(m, n, K, inv_rho, eta_over_rho, seed, warm_iters, bound="power"):
    import torch
    import paper_1705_07112_amd as cpa
    I, _, _ = synth.rpca_frames(m, n, rank=min(40, m // 4), outlier_frac=0.05, seed=seed)
    Id = torch.from_numpy(I).cuda()
    run = cpa.RpcaAdmm(Id, inv_rho, eta_over_rho, cpa.Opts(K=K, warm_start=True, power_iters=100, bound=bound))
    Et = torch.zeros(warm_iters + 1, dtype=torch.float64, device="cuda")
    if warm_iters:
        run.iterate(warm_iters, Et[:warm_iters])
    before = _state_host(run)
    run.iterate(1, Et[warm_iters:])
    torch.cuda.synchronize()
    after = _state_host(run)
    ref, info = drivers.rpca_step(before, I.astype(np.float64), inv_rho, eta_over_rho, K, bound_rule=bound)
    # each dual block is a sum of three terms; its error is measured against the
    # size of those terms (the sum itself can cancel to much less)
    scale = {
        "u1": metrics.fro(before["u1"]) + metrics.fro(ref["l"]) + metrics.fro(ref["z1"]),
        "u2": metrics.fro(before["u2"]) + metrics.fro(ref["s"]) + metrics.fro(ref["z2"]),
        "u3": metrics.fro(before["u3"]) + metrics.fro(ref["l"]) + metrics.fro(ref["s"]) + metrics.fro(I),
    }
    errs = {k: (metrics.fro(after[k] - ref[k]) / scale[k] if k in scale else metrics.rel_fro(after[k], ref[k]))
            for k in NAMES}
    e_gpu = Et[warm_iters].item()
    print(f"  one iteration after {warm_iters}: " + " ".join(f"{k}={v:.2e}" for k, v in errs.items())
          + f" E gpu={e_gpu:.6g} oracle={info['E']:.6g}", flush=True)
    for k in NAMES:
        assert errs[k] <= 1e-5, (k, errs[k])
    assert abs(e_gpu - info["E"]) <= 1e-5 * max(info["E"], 1e-12)


def test_admm_one_iteration_small():
    print("admm 96x80", flush=True)
    _check_one_iteration(96, 80, 20, 1.0, 1.0 / np.sqrt(96), 11, warm_iters=0)
    _check_one_iteration(96, 80, 20, 1.0, 1.0 / np.sqrt(96), 11, warm_iters=6)


def test_admm_one_iteration_odd_width():
    """n % 4 != 0: the pre- and post-steps take their element-by-element path
    (at n % 4 == 0 they move four elements per access)."""
    print("admm 70x53", flush=True)
    _check_one_iteration(70, 53, 20, 1.0, 1.0 / np.sqrt(70), 13, warm_iters=0)
    _check_one_iteration(70, 53, 20, 1.0, 1.0 / np.sqrt(70), 13, warm_iters=5)


@pytest.mark.parametrize("m,n,K,inv_rho,eta,seed", [(96, 80, 20, 1.0, 1.0 / np.sqrt(96), 12),
                                                    (1024, 1024, 30, 10.0, 10.0 / 32.0, synth.BASE_SEED + 1)])
def test_admm_one_iteration_lanczos_bound(m, n, K, inv_rho, eta, seed):
    """The ADMM iteration with the Lanczos bound (one workgroup at d = 80, the
    grid kernel at d = 1024; from the fifth iteration inside the captured graph)."""
    print(f"admm lanczos {m}x{n}", flush=True)
    _check_one_iteration(m, n, K, inv_rho, eta, seed, warm_iters=0, bound="lanczos")
    _check_one_iteration(m, n, K, inv_rho, eta, seed, warm_iters=4, bound="lanczos")


def test_admm_one_iteration_full_size():
    """The bench workload (1024 x 1024, K = 30, 1/rho = 10, eta/rho = 10/32)."""
    print("admm 1024x1024", flush=True)
    _check_one_iteration(1024, 1024, 30, 10.0, 10.0 / 32.0, synth.BASE_SEED + 1, warm_iters=4)


def test_admm_drift_is_small():
    import torch
    import paper_1705_07112_amd as cpa
    m, n, iters = 96, 80, 12
    I, _, _ = synth.rpca_frames(m, n, rank=24, outlier_frac=0.05, seed=11)
    run = cpa.RpcaAdmm(torch.from_numpy(I).cuda(), 1.0, 1.0 / np.sqrt(96), cpa.Opts(K=20, warm_start=True))
    Et = torch.zeros(iters, dtype=torch.float64, device="cuda")
    run.iterate(iters, Et)
    l_o, s_o, E_o, _ = drivers.rpca_admm(I.astype(np.float64), 1.0, 1.0 / np.sqrt(96), iters, 20)
    el = metrics.rel_fro(run.L.cpu().numpy(), l_o)
    es = metrics.rel_fro(run.S.cpu().numpy(), s_o)
    print(f"  drift after {iters}: l {el:.2e} s {es:.2e}", flush=True)
    assert el < 1e-3 and es < 1e-2
    assert np.max(np.abs(Et.cpu().numpy() - np.array(E_o)) / np.array(E_o)) < 1e-2


def test_rpca_one_call_stops_at_tolerance():
    """cpa_rpca_admm: stops at the first iteration with E_t <= tol, and its L, S
    and E_t history equal those of the same number of iterations run with the
    init/iterate pair (cold power bound every iteration, so both runs are the
    same computation)."""
    import torch
    import paper_1705_07112_amd as cpa
    I, _, _ = synth.rpca_frames(96, 80, rank=10, outlier_frac=0.05, seed=31)
    Id = torch.from_numpy(I).cuda()
    opts = cpa.Opts(K=20, warm_start=False, power_iters=100)
    tol = 5e-3
    L, S, E, t = cpa.rpca_admm(Id, 1.0, 1.0 / np.sqrt(96), 300, tol, opts)
    print(f"rpca one call: {t} iterations, E_last={E[-1]:.3e}", flush=True)
    assert 1 < t < 300 and len(E) == t
    assert E[-1] <= tol and all(e > tol for e in E[:-1])
    run = cpa.RpcaAdmm(Id, 1.0, 1.0 / np.sqrt(96), opts)
    Et = torch.zeros(t, dtype=torch.float64, device="cuda")
    run.iterate(t, Et)
    torch.cuda.synchronize()
    assert torch.equal(L, run.L) and torch.equal(S, run.S)
    assert np.array_equal(np.array(E), Et.cpu().numpy())
    # max_iters caps the run
    _, _, E2, t2 = cpa.rpca_admm(Id, 1.0, 1.0 / np.sqrt(96), 3, 0.0, opts)
    assert t2 == 3 and len(E2) == 3


def test_graph_replays_equal_direct_launches():
    """The ADMM iteration replayed from its captured graph equals the same
    iterations launched directly, bit for bit: runs of 5, 4, 2 and 19 replays
    (the last one two replays of the eight-iteration graph and three of the
    one-iteration graph) with synchronisations and eager work between them, each
    run's E_t and the state compared (cold power starts, so neither run depends
    on the other)."""
    import torch
    import paper_1705_07112_amd as cpa
    I, _, _ = synth.rpca_frames(128, 96, rank=12, outlier_frac=0.05, seed=41)
    Id = torch.from_numpy(I).cuda()
    opts = cpa.Opts(K=20, warm_start=False, power_iters=100)
    chunks = (5, 4, 2, 19)
    direct = cpa.RpcaAdmm(Id, 1.0, 1.0 / np.sqrt(128), opts)
    Ed = torch.zeros(sum(chunks), dtype=torch.float64, device="cuda")
    cpa.timing_enable(True)      # per-launch timing forces direct launches
    try:
        direct.iterate(sum(chunks), Ed)
        torch.cuda.synchronize()
    finally:
        cpa.timing_enable(False)
    graphed = cpa.RpcaAdmm(Id, 1.0, 1.0 / np.sqrt(128), opts)
    Eg = torch.zeros(sum(chunks), dtype=torch.float64, device="cuda")
    o = 0
    for c in chunks:
        graphed.iterate(c, Eg[o:o + c])
        torch.cuda.synchronize()
        _ = float((graphed.L * 2.0).sum())   # eager work between the replays
        o += c
    torch.cuda.synchronize()
    print(f"graph vs direct: E_t equal {torch.equal(Ed, Eg)}, state equal {torch.equal(direct.state, graphed.state)}",
          flush=True)
    assert torch.equal(Ed, Eg)
    assert torch.equal(direct.state, graphed.state)
