"""GPU checks of the schedule model kernels (against the float64 reference in oracle.mlp),
the autotuner and the schedule policies (which must never change the bits)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import mlp as ref
from gf2_testutil import run_and_check


@pytest.fixture(scope="module")
def g():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0811_1714_amd as g
    g.lib()
    return g


def split_params(flat, S):
    sizes = [4, 64, 64, 64, S]
    out, off = [], 0
    for fi, fo in zip(sizes[:-1], sizes[1:]):
        out.append(flat[off: off + fi * fo].reshape(fi, fo)); off += fi * fo
        out.append(flat[off: off + fo]); off += fo
    assert off == flat.size
    return out


def test_mlp_forward_backward_adam_match_float64_reference(g):
    import torch
    S = 2 * g.num_candidates()          # latency head and batch-throughput head
    P = g.mlp_param_count()
    assert P == 4 * 64 + 64 + 2 * (64 * 64 + 64) + 64 * S + S
    rng = np.random.default_rng(0)
    batch = 37
    flat = rng.standard_normal(P).astype(np.float32) * 0.3
    X = rng.standard_normal((batch, 4)).astype(np.float32)
    T = rng.standard_normal((batch, S)).astype(np.float32)
    M = (rng.random((batch, S)) < 0.85).astype(np.float32)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    dp, dX, dT, dM = dev(flat), dev(X), dev(T), dev(M)
    dY = torch.empty((batch, S), dtype=torch.float32, device="cuda")
    acts = torch.empty(3 * batch * 64, dtype=torch.float32, device="cuda")
    grads = torch.empty(P, dtype=torch.float32, device="cuda")
    scratch = torch.empty(g.mlp_scratch_floats(batch), dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    print("mlp forward/backward", flush=True)
    g.mlp_forward(dp, dX, dY, acts)
    g.mlp_backward(dp, dX, acts, dY, dT, dM, grads, scratch, loss)
    torch.cuda.synchronize()
    params = [p.astype(np.float64) for p in split_params(flat.astype(np.float64), S)]
    Yr, cache = ref.forward(params, X.astype(np.float64))
    gr = ref.backward(params, cache, Yr, T.astype(np.float64), M.astype(np.float64))
    np.testing.assert_allclose(dY.cpu().numpy(), Yr, rtol=1e-4, atol=1e-4)
    assert abs(loss.item() - ref.loss(Yr, T, M)) <= 1e-4 * max(1.0, ref.loss(Yr, T, M))
    gflat = np.concatenate([x.reshape(-1) for x in gr])
    got = grads.cpu().numpy().astype(np.float64)
    err = np.abs(got - gflat) / (np.abs(gflat) + 1e-3 * np.abs(gflat).max())
    assert err.max() < 1e-3, err.max()
    # One Adam step against the reference.
    m0 = torch.zeros(P, dtype=torch.float32, device="cuda")
    v0 = torch.zeros(P, dtype=torch.float32, device="cuda")
    g.mlp_adam(dp, grads, m0, v0, step=1, lr=1e-2)
    torch.cuda.synchronize()
    newp, _, _ = ref.adam_step([flat.astype(np.float64)], [got], [np.zeros(P)], [np.zeros(P)], 1, lr=1e-2)
    np.testing.assert_allclose(dp.cpu().numpy(), newp[0], rtol=1e-5, atol=1e-6)
    # argmin with a mask
    allowed = torch.zeros(S, dtype=torch.uint8, device="cuda")
    allowed[[1, 3, 5, 13]] = 1
    out = torch.empty(batch, dtype=torch.int32, device="cuda")
    g.mlp_argmin(dY, out, allowed)
    y = dY.cpu().numpy()
    sub = np.array([1, 3, 5, 13])
    assert np.array_equal(out.cpu().numpy(), sub[np.argmin(y[:, sub], axis=1)])


def test_autotune_and_policies_keep_bits(g):
    print("autotune", flush=True)
    ms, best = g.autotune(700, 900, 1100, density=0.3, reps=2)
    assert ms.shape == (g.num_candidates(),) and 0 <= best < ms.size and ms[best] > 0
    assert ms[best] == ms[ms > 0].min()
    mb, bb, copies = g.autotune_batch(300, 500, 700, density=0.5, reps=2)
    assert copies >= 2 and 0 <= bb < mb.size and mb[bb] > 0 and (mb > 0).sum() >= 7
    # Partial re-timing: only the listed candidates get a time, alone or inside a batch.
    sub = [7, 0, 28]
    for batch in (False, True):
        ps, pc = g.autotune_candidates(300, 500, 700, sub, density=0.5, reps=2, batch=batch)
        assert (ps[sub] > 0).all() and (np.delete(ps, sub) == -1).all()
        assert (pc >= 2) if batch else (pc == 1)
    try:
        base = run_and_check(g, 700, 900, 1100, seed=41)
        g.set_policy(g.POLICY_AUTOTUNE)
        assert np.array_equal(run_and_check(g, 700, 900, 1100, seed=41), base)
        rng = np.random.default_rng(1)
        g.set_model(rng.standard_normal(g.mlp_param_count()).astype(np.float32),
                    np.array([9, 9, 9, .25, 2, 2, 2, .2], dtype=np.float32))
        g.set_policy(g.POLICY_MODEL)
        assert np.array_equal(run_and_check(g, 700, 900, 1100, seed=41), base)
        c = g.choose_schedule(700, 900, 1100, batch=True)
        assert 0 <= c < g.num_candidates()
    finally:
        g.set_policy(g.POLICY_FIXED)
        g.set_model(None)


def test_trained_model_gain_over_fixed_heuristic_on_fresh_shapes(g):
    """What the trained network gains over the method without it.  On 128 shapes it never
    saw (the batch workload's shape law, a seed disjoint from training and held-out data),
    every candidate the persistent batch kernel can run is timed per product inside a batch
    of copies (exhaustive autotune, the yardstick for regret).  The model's pick (batch head)
    must be within 10% of the fastest on average and strictly better on average than the
    fixed heuristic (the analytic tile-height rule), which is what the library does without it."""
    import os
    import synth
    if not os.path.exists(g.DEFAULT_MODEL):
        pytest.skip("no trained model")
    dims = synth.log_uniform_dims(77, 5, 128, 64, 4096)
    dens = synth.log_uniform_p(77, 1005, 128, 0.01, 0.5)
    allowed = np.array([g.batch_candidate(i) for i in range(g.num_candidates())])
    r_model, r_fixed = [], []
    try:
        g.load_model()
        for (m, k, n), p in zip(dims, dens):
            m, k, n = int(m), int(k), int(n)
            ms, _, _ = g.autotune_batch(m, k, n, density=float(p), reps=3)
            t = np.where(allowed & (ms > 0), ms, np.inf)
            g.set_policy(g.POLICY_MODEL)
            pick_model = g.choose_schedule(m, k, n, batch=True)
            g.set_policy(g.POLICY_FIXED)
            pick_fixed = g.choose_schedule(m, k, n, batch=True)
            r_model.append(t[pick_model] / t.min() - 1)
            r_fixed.append(t[pick_fixed] / t.min() - 1)
            print(f"{(m, k, n)} model {pick_model} fixed {pick_fixed} regret {r_model[-1]:.3f} / {r_fixed[-1]:.3f}",
                  flush=True)
    finally:
        g.set_policy(g.POLICY_FIXED)
        g.set_model(None)
    mean_model, mean_fixed = float(np.mean(r_model)), float(np.mean(r_fixed))
    print(f"mean regret: model {mean_model:.4f}, fixed heuristic {mean_fixed:.4f}", flush=True)
    assert mean_model <= 0.10
    assert mean_model < mean_fixed


def test_model_planned_batch_beats_fixed_heuristic_batch(g):
    """End to end on a fresh uneven batch (4096 products, m, k, n log-uniform in [64, 4096), a seed
    disjoint from the training data): the plan whose schedules the trained model chose runs
    faster than the plan the fixed heuristic chose, and both give the same bits.  The two plans
    are replayed alternately (15 times each, after warm-up) so that clock drift affects both
    alike; their medians are compared."""
    import os
    import torch
    import synth
    if not os.path.exists(g.DEFAULT_MODEL):
        pytest.skip("no trained model")
    count = 4096
    dims = synth.log_uniform_dims(91, 4, count, 64, 4096)
    W = lambda c: (int(c) + 63) // 64
    sizes = [int(m) * W(k) + int(k) * W(n) for m, k, n in dims]
    csz = [int(m) * W(n) for m, k, n in dims]
    ioff = np.concatenate([[0], np.cumsum([(x + 31) // 32 * 32 for x in sizes])])
    coff = np.concatenate([[0], np.cumsum([(x + 31) // 32 * 32 for x in csz])])
    gen = torch.Generator(device="cuda").manual_seed(91)
    pool = torch.randint(-(1 << 62), 1 << 62, (int(ioff[-1]),), dtype=torch.int64, device="cuda", generator=gen)
    plans, outs = {}, {}
    try:
        g.load_model()
        for policy in (g.POLICY_FIXED, g.POLICY_MODEL):
            g.set_policy(policy)
            cpool = torch.zeros(int(coff[-1]), dtype=torch.int64, device="cuda")
            plist = []
            for i, (m, k, n) in enumerate(dims):
                m, k, n = int(m), int(k), int(n)
                b = int(ioff[i])
                A = pool[b: b + m * W(k)].view(m, W(k))
                B = pool[b + m * W(k): b + sizes[i]].view(k, W(n))
                C = cpool[int(coff[i]): int(coff[i]) + csz[i]].view(m, W(n))
                plist.append(g.problem(C, A, B, m, k, n))
            print(f"plan of {count} products under policy {policy}", flush=True)
            plans[policy] = g.BatchPlan(plist)
            outs[policy] = cpool
        times = {p: [] for p in plans}
        for _ in range(3):
            for p in plans:
                plans[p].execute()
        torch.cuda.synchronize()
        for _ in range(15):
            for p, plan in plans.items():
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                plan.execute()
                e1.record()
                torch.cuda.synchronize()
                times[p].append(e0.elapsed_time(e1))
    finally:
        for plan in plans.values():
            plan.destroy()
        g.set_policy(g.POLICY_FIXED)
        g.set_model(None)
    t_fixed, t_model = float(np.median(times[g.POLICY_FIXED])), float(np.median(times[g.POLICY_MODEL]))
    print(f"batch ms (median of 15): fixed {t_fixed:.3f}, model {t_model:.3f}", flush=True)
    assert torch.equal(outs[g.POLICY_FIXED], outs[g.POLICY_MODEL]), "the two plans gave different bits"
    assert t_model < t_fixed
