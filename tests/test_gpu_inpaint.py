"""GPU texture-inpainting ADMM (Appendix A, eq. admm_algorithm_inp) against the
oracle driver.

Gated: one iteration started from the same state on both sides (the GPU's own
state, copied to the host) must agree to the FP32 tolerance, every block of
[l, z1..z5, u1..u5]; each dual block's error is measured against the size of
the terms it sums.  Then the recovery of a low-rank texture's missing block
with the pin's parameters.  The scheduled driver (z1 by the sparsified shrink
with the DCT, keep from eq. recommendation_epsilon) is gated the same way for
each of the schedule's three cases, where the oracle's |Phi| has a clear gap at
the keep count (so FP32 and FP64 keep the same entries), and over a run whose
keep sequence must match the oracle's exactly."""
import math

import numpy as np
import pytest

import synth
from oracle import drivers, metrics, sparsify

pytestmark = pytest.mark.gpu

NAMES = drivers.INPAINT_NAMES


def _state_host(run):
    return {k: run.block(i).cpu().numpy().astype(np.float64) for i, k in enumerate(NAMES)}


def _run(m, n, hole, border_w, with_mean, K, inv_rho, eta, seed, bound="power"):
    import torch
    import paper_1705_07112_amd as cpa
    I, om, bd, L0 = synth.texture(m, n, hole=hole, border=border_w, seed=seed)
    Id = torch.from_numpy(I.astype(np.float32)).cuda()
    run = cpa.Inpaint(Id, torch.from_numpy(om), inv_rho, eta,
                      cpa.Opts(K=K, warm_start=True, power_iters=100, bound=bound),
                      border=torch.from_numpy(bd.astype(np.float32)) if with_mean else None)
    return run, I.astype(np.float32).astype(np.float64), om, bd, L0


@pytest.mark.parametrize("bound", ["power", "lanczos"])
@pytest.mark.parametrize("with_mean", [True, False])
@pytest.mark.parametrize("shape,hole", [((96, 80), (30, 60, 20, 44)), ((130, 70), (40, 71, 9, 33))])
def test_inpaint_one_iteration(shape, hole, with_mean, bound):
    import torch
    m, n = shape
    K, inv_rho, eta = 20, 1.0, 0.01
    run, I, om, bd, _ = _run(m, n, hole, 3, with_mean, K, inv_rho, eta, 8100 + m, bound)
    for warm in (0, 6):
        if warm:
            run.iterate(warm)
        before = _state_host(run)
        Et = torch.zeros(1, dtype=torch.float64, device="cuda")
        run.iterate(1, Et)
        torch.cuda.synchronize()
        after = _state_host(run)
        ref, info = drivers.inpaint_step(before, I, om, bd if with_mean else None, inv_rho, eta, K, bound_rule=bound)
        P = drivers.dct2(ref["l"])
        scale = {"u1": metrics.fro(before["u1"]) + metrics.fro(ref["l"]) + metrics.fro(ref["z1"]),
                 "u2": metrics.fro(before["u2"]) + metrics.fro(P) + metrics.fro(ref["z2"]),
                 "u3": metrics.fro(before["u3"]) + metrics.fro(om * ref["l"]) + metrics.fro(ref["z3"]),
                 "u4": metrics.fro(before["u4"]) + metrics.fro(ref["l"]) + metrics.fro(ref["z4"]),
                 "u5": metrics.fro(before["u5"]) + metrics.fro((1 - om) * ref["l"]) + metrics.fro(ref["z5"])}
        errs = {k: (metrics.fro(after[k] - ref[k]) / scale[k] if k in scale else metrics.rel_fro(after[k], ref[k]))
                for k in NAMES}
        print(f"inpaint {m}x{n} mean={with_mean} after {warm}: " + " ".join(f"{k}={v:.1e}" for k, v in errs.items())
              + f" E gpu={Et.item():.6g} oracle={info['E']:.6g}", flush=True)
        for k in NAMES:
            assert errs[k] <= 1e-5, (k, errs[k])
        assert abs(Et.item() - info["E"]) <= 1e-5 * max(info["E"], 1e-12)


def test_inpaint_recovers_a_low_rank_texture():
    """The oracle pin's problem (48 x 40, 12 x 10 hole, 120 iterations): E_t falls
    below 1e-4 and the hole is recovered to 25%, like the oracle's run."""
    import torch
    run, I, om, bd, L0 = _run(48, 40, None, 4, True, 20, 1.0, 0.01, 5)
    Et = torch.zeros(120, dtype=torch.float64, device="cuda")
    run.iterate(120, Et)
    torch.cuda.synchronize()
    l = run.L.cpu().numpy().astype(np.float64)
    reg = om == 0.0
    err = np.linalg.norm((l - L0)[reg]) / np.linalg.norm(L0[reg])
    l_o, E_o = drivers.inpaint_admm(I, om, bd, 1.0, 0.01, 120, 20)
    err_o = np.linalg.norm((l_o - L0)[reg]) / np.linalg.norm(L0[reg])
    print(f"inpaint recovery: hole err gpu {err:.4f} oracle {err_o:.4f}; E_t gpu {Et[-1].item():.2e} "
          f"oracle {E_o[-1]:.2e}; drift {metrics.rel_fro(l, l_o):.2e}", flush=True)
    assert Et[-1].item() < 1e-4
    assert err < 0.25
    assert abs(err - err_o) <= 0.01


def _errs(before, after, ref, om):
    P = drivers.dct2(ref["l"])
    scale = {"u1": metrics.fro(before["u1"]) + metrics.fro(ref["l"]) + metrics.fro(ref["z1"]),
             "u2": metrics.fro(before["u2"]) + metrics.fro(P) + metrics.fro(ref["z2"]),
             "u3": metrics.fro(before["u3"]) + metrics.fro(om * ref["l"]) + metrics.fro(ref["z3"]),
             "u4": metrics.fro(before["u4"]) + metrics.fro(ref["l"]) + metrics.fro(ref["z4"]),
             "u5": metrics.fro(before["u5"]) + metrics.fro((1 - om) * ref["l"]) + metrics.fro(ref["z5"])}
    return {k: (metrics.fro(after[k] - ref[k]) / scale[k] if k in scale else metrics.rel_fro(after[k], ref[k]))
            for k in NAMES}


def _clear_gap(x, T, keep, rel=1e-4):
    """|Phi| of the shrink input has its keep-th value at least rel * max|Phi| away
    from every other distinct magnitude (equal magnitudes: the mirrored entries)."""
    Phi, _ = sparsify.transformed_gram(x, T)
    a = np.sort(np.abs(Phi).ravel())[::-1]
    eps = a[keep - 1]
    tie = np.abs(a - eps) <= 1e-12 * a[0]
    others = a[~tie]
    return others.size == 0 or float(np.min(np.abs(others - eps))) > rel * a[0]


@pytest.mark.parametrize("E_prev", [1.0, 0.01, 1e-4])
def test_scheduled_inpaint_one_iteration_each_case(E_prev):
    import torch
    m, n, K, inv_rho, eta = 256, 192, 15, 1.0, 0.01
    run, I, om, bd, _ = _run(m, n, None, 4, True, K, inv_rho, eta, 5)
    T = sparsify.dct_matrix(n)
    keep_o = sparsify.keep_schedule(E_prev, n)
    # from the start state the shrink input is nearly constant and Phi nearly rank
    # one: its k-th magnitude is rounding noise, so the gated states come later
    done = 0
    for warm in (3, 3):
        run.iterate(warm)
        done += warm
        before = _state_host(run)
        saved = run.state.clone()
        Et = torch.zeros(1, dtype=torch.float64, device="cuda")
        keeps = run.iterate_scheduled(1, Et, transform="dct", E_prev=E_prev)
        torch.cuda.synchronize()
        after = _state_host(run)
        run.state.copy_(saved)
        ref, info = drivers.inpaint_step(before, I, om, bd, inv_rho, eta, K, sparsify={"T": T, "keep": keep_o})
        assert _clear_gap(info["x"], T, keep_o), "data: no clear gap at the keep count"
        errs = _errs(before, after, ref, om)
        print(f"scheduled inpaint E_prev={E_prev} after {done}: keep gpu {keeps[0]} oracle {keep_o}; "
              + " ".join(f"{k}={v:.1e}" for k, v in errs.items()) + f" E gpu={Et.item():.6g} oracle={info['E']:.6g}",
              flush=True)
        assert keeps == [keep_o]
        for k in NAMES:
            assert errs[k] <= 1e-5, (k, errs[k])
        assert abs(Et.item() - info["E"]) <= 1e-5 * max(info["E"], 1e-12)


def test_scheduled_inpaint_run_follows_the_oracle():
    """24 iterations from the start (E_prev = +inf) with the paper's switch points:
    the keep moves from k_1 to k_2 as E_t falls below E_l; both sides take the same
    keeps, E_t agrees and the final image drifts by FP32 rounding only."""
    import torch
    m = n = 256
    K, inv_rho, eta, iters = 15, 1.0, 0.01, 24
    run, I, om, bd, L0 = _run(m, n, None, 4, True, K, inv_rho, eta, 5)
    Et = torch.zeros(iters, dtype=torch.float64, device="cuda")
    keeps = run.iterate_scheduled(iters, Et, transform="dct")
    torch.cuda.synchronize()
    l = run.L.cpu().numpy().astype(np.float64)
    st, E_o, keeps_o = drivers.inpaint_admm(I, om, bd, inv_rho, eta, iters, K,
                                            schedule={"T": sparsify.dct_matrix(n), "E_prev": math.inf})
    # the oracle's E_t stay clear of the switch points, so FP32 drift cannot flip a keep
    assert all(abs(e - 0.03) > 0.01 * 0.03 and abs(e - 6e-4) > 0.01 * 6e-4 for e in E_o)
    E_g = Et.cpu().numpy()
    dE = float(np.max(np.abs(E_g - np.array(E_o)) / np.maximum(np.array(E_o), 1e-12)))
    drift = metrics.rel_fro(l, st["l"])
    reg = om == 0.0
    err = np.linalg.norm((l - L0)[reg]) / np.linalg.norm(L0[reg])
    err_o = np.linalg.norm((st["l"] - L0)[reg]) / np.linalg.norm(L0[reg])
    print(f"scheduled inpaint run: keeps gpu {keeps} oracle {keeps_o}; max rel dE {dE:.2e}; drift {drift:.2e}; "
          f"hole err gpu {err:.4f} oracle {err_o:.4f}", flush=True)
    assert keeps == keeps_o
    assert len(set(keeps)) == 2
    assert dE <= 1e-3
    assert drift <= 1e-3


def test_scheduled_inpaint_continues_across_calls():
    """16 iterations in one call equal 8 + 8 with the second call given the first's
    last E_t as E_prev, bit for bit (the same keeps, E_t and state).  The power
    bound starts cold in every shrink here, so the two runs do not share a warm
    start through the context."""
    import torch
    import paper_1705_07112_amd as cpa
    m, n = 128, 96
    I, om, bd, _ = synth.texture(m, n, border=4, seed=5)
    runs = []
    for split in (False, True):
        run = cpa.Inpaint(torch.from_numpy(I.astype(np.float32)).cuda(), torch.from_numpy(om), 1.0, 0.01,
                          cpa.Opts(K=15, warm_start=False, power_iters=100),
                          border=torch.from_numpy(bd.astype(np.float32)))
        Et = torch.zeros(16, dtype=torch.float64, device="cuda")
        if split:
            keeps = run.iterate_scheduled(8, Et[:8], transform="dct")
            torch.cuda.synchronize()
            keeps += run.iterate_scheduled(8, Et[8:], transform="dct", E_prev=Et[7].item())
        else:
            keeps = run.iterate_scheduled(16, Et, transform="dct")
        torch.cuda.synchronize()
        runs.append((keeps, Et.cpu().numpy(), run.state.cpu().numpy()))
    (k1, e1, s1), (k2, e2, s2) = runs
    print(f"scheduled inpaint split run: keeps {k1}", flush=True)
    assert k1 == k2
    assert np.array_equal(e1, e2)
    assert np.array_equal(s1, s2)


def test_scheduled_inpaint_rejects_a_gram_side_off_the_8_grid():
    """The sparsified shrink needs a Gram side that is a multiple of 8: the
    scheduled driver says so before any work is queued, and the state is unchanged."""
    import torch
    import paper_1705_07112_amd as cpa
    run, *_ = _run(100, 90, (40, 60, 30, 50), 3, True, 12, 1.0, 0.01, 7)
    before = run.state.clone()
    Et = torch.zeros(2, dtype=torch.float64, device="cuda")
    with pytest.raises(cpa.CpaError) as e:
        run.iterate_scheduled(2, Et, transform="dct")
    assert e.value.status == 2 and "multiple of 8" in str(e.value)
    torch.cuda.synchronize()
    assert torch.equal(run.state, before)


def test_inpaint_one_iteration_full_size():
    """The bench's inpainting workload at full size (2560 x 1920, 300 x 300 hole,
    8-pixel frame, K = 20, 1/rho = 6, eta/rho = 0.1): one iteration from the GPU's
    own state after two, every block against the oracle step."""
    import torch
    m, n, K, inv_rho, eta = 2560, 1920, 20, 6.0, 0.1
    hole = (m // 2 - 150, m // 2 + 150, n // 2 - 150, n // 2 + 150)
    I, om, bd, _ = synth.texture(m, n, terms=4, hole=hole, border=8, seed=synth.BASE_SEED + 7)
    import paper_1705_07112_amd as cpa
    run = cpa.Inpaint(torch.from_numpy(I.astype(np.float32)).cuda(), torch.from_numpy(om), inv_rho, eta,
                      cpa.Opts(K=K, warm_start=True, power_iters=100), border=torch.from_numpy(bd.astype(np.float32)))
    run.iterate(2)
    before = _state_host(run)
    Et = torch.zeros(1, dtype=torch.float64, device="cuda")
    run.iterate(1, Et)
    torch.cuda.synchronize()
    after = _state_host(run)
    ref, info = drivers.inpaint_step(before, I.astype(np.float32).astype(np.float64), om, bd, inv_rho, eta, K)
    errs = _errs(before, after, ref, om)
    print("inpaint 2560x1920 one iteration: " + " ".join(f"{k}={v:.1e}" for k, v in errs.items())
          + f" E gpu={Et.item():.6g} oracle={info['E']:.6g}", flush=True)
    for k in NAMES:
        assert errs[k] <= 1e-5, (k, errs[k])
    assert abs(Et.item() - info["E"]) <= 1e-5 * max(info["E"], 1e-12)
