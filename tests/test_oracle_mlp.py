"""Pins for the float64 schedule-model reference (no GPU).

Gradients are checked by central finite differences (not by retyping the chain
rule); Adam by its closed-form first step and by convergence on a quadratic.
"""
import numpy as np

from oracle import mlp


def make_batch(seed, n=16, nin=4, nout=6):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, nin))
    T = rng.standard_normal((n, nout))
    M = (rng.random((n, nout)) < 0.8).astype(np.float64)
    return X, T, M


def test_gradients_match_central_finite_differences():
    sizes = [4, 7, 5, 6, 6]
    params = mlp.init_params(sizes, seed=3)
    for i in range(1, len(params), 2):       # non-zero biases so no unit sits exactly at the ReLU kink
        params[i] = np.random.default_rng(i).standard_normal(params[i].shape) * 0.1
    X, T, M = make_batch(1, nout=6)
    Y, cache = mlp.forward(params, X)
    grads = mlp.backward(params, cache, Y, T, M)
    h = 1e-6
    rng = np.random.default_rng(0)
    for pi, p in enumerate(params):
        flat = p.reshape(-1)
        for idx in rng.choice(flat.size, size=min(flat.size, 12), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = mlp.loss(mlp.forward(params, X)[0], T, M)
            flat[idx] = old - h
            lm = mlp.loss(mlp.forward(params, X)[0], T, M)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = grads[pi].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 + 1e-5 * abs(fd), (pi, idx, fd, an)


def test_output_bias_gradient_closed_form_with_zero_weights():
    sizes = [4, 8, 8, 3]
    params = [np.zeros_like(p) for p in mlp.init_params(sizes)]
    params[-1] = np.array([0.5, -1.0, 2.0])
    X, T, M = make_batch(2, nout=3)
    Y, cache = mlp.forward(params, X)
    assert np.allclose(Y, params[-1])
    g = mlp.backward(params, cache, Y, T, M)
    expect = 2 * ((params[-1] - T) * M).sum(axis=0) / M.sum()
    assert np.allclose(g[-1], expect)
    assert all(np.all(gi == 0) for gi in g[:-2])   # dead ReLUs pass no gradient further down


def test_adam_first_step_is_lr_times_sign():
    p = [np.array([1.0, -2.0, 3.0])]
    g = [np.array([0.3, -5.0, 1e-3])]
    z = [np.zeros(3)]
    newp, _, _ = mlp.adam_step(p, g, z, z, t=1, lr=0.01, eps=1e-12)
    assert np.allclose(newp[0], p[0] - 0.01 * np.sign(g[0]))


def test_adam_minimises_a_quadratic_and_training_reduces_loss():
    p = [np.array([5.0, -3.0])]
    m = [np.zeros(2)]
    v = [np.zeros(2)]
    for t in range(1, 3001):
        p, m, v = mlp.adam_step(p, [2 * p[0]], m, v, t, lr=0.05)
    assert np.all(np.abs(p[0]) < 1e-2)
    sizes = [4, 16, 16, 3]
    params = mlp.init_params(sizes, seed=1)
    X, T, M = make_batch(3, n=64, nout=3)
    mo = [np.zeros_like(q) for q in params]
    vo = [np.zeros_like(q) for q in params]
    l0 = mlp.loss(mlp.forward(params, X)[0], T, M)
    for t in range(1, 301):
        Y, c = mlp.forward(params, X)
        params, mo, vo = mlp.adam_step(params, mlp.backward(params, c, Y, T, M), mo, vo, t, lr=1e-2)
    assert mlp.loss(mlp.forward(params, X)[0], T, M) < 0.5 * l0


def test_committed_schedule_model_regret_recomputed():
    """The committed schedule model against the committed timing set, recomputed here rather
    than read from the training report: the held-out shapes' per-product batch timings of every
    candidate (exhaustive autotuning, the yardstick), the model's batch-head pick from the
    float64 forward pass of this module with the committed weights and feature normalisation,
    and the fixed heuristic's pick from the library (GF2_POLICY_FIXED, host code).  The model
    must be within 10% of the fastest candidate on average and strictly better on average than
    the fixed heuristic, both by its argmin and under the library's batch rule (the model's pick
    only where predicted at least 10% faster than the fixed rule's); the training set must hold
    at least 6000 timed shapes."""
    import os
    import paper_0811_1714_amd as g
    tune = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_0811_1714_amd", "tune")
    model = np.load(os.path.join(tune, "schedule_model.npz"))
    parts = [np.load(os.path.join(tune, f)) for f in sorted(os.listdir(tune)) if f.startswith("timings_mi355x_")]
    assert sum(len(q["train_dims"]) for q in parts) >= 6000
    ho = [q for q in parts if len(q["heldout_dims"])]
    assert len(ho) == 1 and len(ho[0]["heldout_dims"]) == 500
    dims, dens, ms = ho[0]["heldout_dims"], ho[0]["heldout_density"], ho[0]["heldout_ms"].astype(np.float64)
    S = g.num_candidates()
    assert ms.shape[1] == 2 * S and model["target_mean"].size == 2 * S
    sizes = [4, 64, 64, 64, 2 * S]
    flat, params, off = model["params"].astype(np.float64), [], 0
    for fi, fo in zip(sizes[:-1], sizes[1:]):
        params.append(flat[off: off + fi * fo].reshape(fi, fo)); off += fi * fo
        params.append(flat[off: off + fo]); off += fo
    assert off == flat.size
    norm = model["norm"].astype(np.float64)
    X = (np.column_stack([np.log2(dims.astype(np.float64)), dens.astype(np.float64)]) - norm[:4]) / norm[4:]
    Y = mlp.forward(params, X)[0]
    allowed = np.array([g.batch_candidate(i) for i in range(S)])
    t = np.where(allowed[None, :] & (ms[:, S:] > 0), ms[:, S:], np.inf)
    pick_model = np.where(allowed[None, :], Y[:, S:], np.inf).argmin(axis=1)
    pol = g.get_policy()
    g.set_policy(g.POLICY_FIXED)
    try:
        pick_fixed = np.array([g.choose_schedule(int(m), int(k), int(n), batch=True) for m, k, n in dims])
    finally:
        g.set_policy(pol)
    rows = np.arange(len(t))
    # The library's batch rule: the model's pick replaces the fixed rule's only where its
    # predicted time (the outputs are natural-log milliseconds) is at least 10% lower.
    keep = Y[rows, S + pick_model] - Y[rows, S + pick_fixed] < np.log(0.9)
    pick_rule = np.where(keep, pick_model, pick_fixed)
    r_model = t[rows, pick_model] / t.min(axis=1) - 1
    r_rule = t[rows, pick_rule] / t.min(axis=1) - 1
    r_fixed = t[rows, pick_fixed] / t.min(axis=1) - 1
    assert np.isfinite(r_model).all() and np.isfinite(r_fixed).all() and np.isfinite(r_rule).all()
    assert r_model.mean() <= 0.10 and r_rule.mean() <= 0.10
    assert r_model.mean() < r_fixed.mean(), (r_model.mean(), r_fixed.mean())
    assert r_rule.mean() < r_fixed.mean(), (r_rule.mean(), r_fixed.mean())


def test_library_batch_rule_matches_its_definition():
    """Under the model policy the library's batch pick (host inference, ``gf2_choose_schedule``)
    is the batch head's argmin over the persistent-kernel candidates where that is predicted at
    least 10% faster than the fixed rule's candidate, else the fixed rule's candidate.  Recomputed
    here with the float64 forward pass on 300 fresh shapes; a disagreement is allowed only where
    float32 and float64 could round differently (a near-tie in the argmin or at the margin)."""
    import os
    import paper_0811_1714_amd as g
    if not os.path.exists(g.DEFAULT_MODEL):
        pytest.skip("no trained model")
    model = np.load(g.DEFAULT_MODEL)
    S = g.num_candidates()
    sizes = [4, 64, 64, 64, 2 * S]
    flat, params, off = model["params"].astype(np.float64), [], 0
    for fi, fo in zip(sizes[:-1], sizes[1:]):
        params.append(flat[off: off + fi * fo].reshape(fi, fo)); off += fi * fo
        params.append(flat[off: off + fo]); off += fo
    norm = model["norm"].astype(np.float64)
    rng = np.random.default_rng(2024)
    dims = np.exp(rng.uniform(np.log(64), np.log(4096), (300, 3))).astype(np.int64)
    X = (np.column_stack([np.log2(dims.astype(np.float64)), np.full(len(dims), 0.5)]) - norm[:4]) / norm[4:]
    Y = mlp.forward(params, X)[0][:, S:]
    allowed = np.array([g.batch_candidate(i) for i in range(S)])
    pol = g.get_policy()
    try:
        g.set_policy(g.POLICY_FIXED)
        fixed = np.array([g.choose_schedule(int(m), int(k), int(n), batch=True) for m, k, n in dims])
        g.load_model()
        g.set_policy(g.POLICY_MODEL)
        lib_pick = np.array([g.choose_schedule(int(m), int(k), int(n), batch=True) for m, k, n in dims])
    finally:
        g.set_policy(pol)
        g.set_model(None)
    rows = np.arange(len(dims))
    Ya = np.where(allowed[None, :], Y, np.inf)
    arg = Ya.argmin(axis=1)
    margin = Y[rows, arg] - Y[rows, fixed] - np.log(0.9)
    want = np.where(margin < 0, arg, fixed)
    second = np.sort(Ya, axis=1)[:, 1]
    near = (np.abs(margin) < 1e-4) | (second - Ya[rows, arg] < 1e-4)
    bad = (lib_pick != want) & ~near
    assert not bad.any(), [(tuple(dims[i]), lib_pick[i], want[i]) for i in np.flatnonzero(bad)[:5]]
    assert (want != fixed).sum() >= 10          # the rule does depart from the fixed heuristic
    assert (want == fixed).sum() >= 10          # ... and does keep it
