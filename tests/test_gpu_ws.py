"""GPU parity of the learned warm start (BF16 matrix-core MLP, feature and
target rows, start scatter, cold-restart fallback) against the FP64 oracle.

Bars.  The kernels use BF16 weights, BF16 feature rows and BF16
back-propagated deltas, keep the hidden activations as BF16 hi / lo pairs
(about 16 significant bits) and accumulate in FP32.  The oracle is the plain
FP64 definition, run on the same BF16-rounded weights and inputs.  What
separates the two is the BF16 rounding of each delta (about 2e-3 relative on
the first layer's weight gradient), the activations' pair rounding and FP32
accumulation order: relative Frobenius error 1e-2 for every gradient and
the forward output, 1e-3 for the loss.  Adam is checked on the kernel's own
gradient (FP32 vs FP64 arithmetic: 1e-5).  Feature rows are BF16 roundings
of FP32 sums: 1e-2 relative + 1e-3 absolute.  Target rows are FP32
conversions of the solver's FP64 state: 1e-6 relative.
"""
import numpy as np
import pytest

from oracle import mlp as OM
from paper_2604_07644_amd import workloads as W

pytestmark = pytest.mark.gpu

from paper_2604_07644_amd import gsls  # noqa: E402  (fails loudly without libgsls.so)
import torch  # noqa: E402


def _bf16_round(a):
    return torch.tensor(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).float().numpy().astype(np.float64)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def _model(seed=0):
    th = W.ws_init(seed)
    sk = W.ws_sketch()
    return gsls.WarmStart(th.astype(np.float32), sk.astype(np.float32)), th, sk


def _rows(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, 160)) * 0.8
    T = rng.standard_normal((n, 192))
    M = (rng.random((n, 192)) < 0.6).astype(np.float64)
    return X, T, M


def _dev(a, dtype):
    return torch.tensor(np.asarray(a), dtype=dtype, device="cuda")


def test_forward_matches_oracle_ragged_rows():
    ws, th, _ = _model(1)
    X, _, _ = _rows(333, 2)                      # 5 full 64-row tiles and a ragged one
    Xd = _dev(X, torch.float32).to(torch.bfloat16)
    Y = ws.forward(Xd).cpu().numpy()
    thb = _bf16_round(th)                        # the kernels use BF16 weights, FP32 biases
    biases = np.zeros_like(th, dtype=bool)
    o = 0
    for a, b in zip(OM.SIZES[:-1], OM.SIZES[1:]):
        o += a * b
        biases[o:o + b] = True
        o += b
    thb[biases] = th[biases].astype(np.float32)
    Xb = Xd.float().cpu().numpy()
    ref64, _ = OM.forward(thb, Xb)
    assert _rel(Y, ref64) < 1e-2, _rel(Y, ref64)
    ws.close()


def test_gradient_matches_oracle_with_row_gather():
    ws, th, _ = _model(3)
    X, T, M = _rows(1100, 4)                     # gathered rows span three 512-row chunks
    perm = np.random.default_rng(5).permutation(1100)[:777].astype(np.int32)
    Xd = _dev(X, torch.float32).to(torch.bfloat16)
    Td, Md = _dev(T, torch.float32), _dev(M, torch.float32)
    idx = _dev(perm, torch.int32)
    loss, g = ws.loss_grad(Xd, Td, Md, idx=idx)
    thb = _bf16_round(th)
    Xs = Xd.float().cpu().numpy()[perm]
    refL, refg = OM.loss_grad(thb, Xs, T[perm], M[perm])
    assert abs(loss - refL) <= 1e-3 * refL, (loss, refL)
    o = 0
    for li, (a, b) in enumerate(zip(OM.SIZES[:-1], OM.SIZES[1:])):
        gw, rw = g[o:o + a * b], refg[o:o + a * b]; o += a * b
        gb, rb = g[o:o + b], refg[o:o + b]; o += b
        print(f"layer {li}: W {_rel(gw, rw):.2e}  b {_rel(gb, rb):.2e}")
        assert _rel(gw, rw) < 1e-2, (li, "W", _rel(gw, rw))
        assert _rel(gb, rb) < 1e-2, (li, "b", _rel(gb, rb))
    ws.close()


def test_adam_step_matches_oracle_on_kernel_gradient():
    ws, th, _ = _model(6)
    X, T, M = _rows(256, 7)
    Xd = _dev(X, torch.float32).to(torch.bfloat16)
    Td, Md = _dev(T, torch.float32), _dev(M, torch.float32)
    _, g = ws.loss_grad(Xd, Td, Md)
    p0 = ws.params().astype(np.float64)
    ws.train_step(Xd, Td, Md, lr=1e-3)
    p1 = ws.params().astype(np.float64)
    ref, _, _ = OM.adam(p0, g.astype(np.float64), np.zeros_like(p0), np.zeros_like(p0), 1, lr=1e-3)
    np.testing.assert_allclose(p1, ref, rtol=1e-5, atol=1e-7)
    ws.close()


def test_training_lowers_loss():
    ws, _, _ = _model(8)
    X, _, M = _rows(2048, 9)
    # a learnable target: a fixed linear map of the inputs
    A = np.random.default_rng(10).standard_normal((160, 192)) / np.sqrt(160)
    Xd = _dev(X, torch.float32).to(torch.bfloat16)
    T = Xd.float().cpu().numpy() @ A
    Td, Md = _dev(T, torch.float32), _dev(M, torch.float32)
    l0, _ = ws.loss_grad(Xd, Td, Md)
    for _ in range(150):
        ws.train_step(Xd, Td, Md, lr=1e-3)
    l1, _ = ws.loss_grad(Xd, Td, Md)
    assert l1 < 0.2 * l0, (l0, l1)
    ws.close()


def _box_batch():
    return W.uneven_batch(count=6, cfg_id=43, nmin=16, nmax=40)


def test_feature_rows_match_oracle():
    ws, _, sk = _model(11)
    probs = _box_batch()
    b = gsls.Batch(probs)
    X = ws.features(b).float().cpu().numpy()
    ref = np.concatenate([OM.features(p, sk) for p in probs])
    assert X.shape == ref.shape == (b.rows(), 160)
    np.testing.assert_allclose(X, ref, rtol=1e-2, atol=1e-3)
    b.close(); ws.close()


def test_target_rows_match_oracle():
    probs = _box_batch()
    b = gsls.Batch(probs)
    res, _ = b.solve(tol=1e-5)
    T, M = gsls.WarmStart.targets(b)
    T, M = T.cpu().numpy(), M.cpu().numpy()
    o = 0
    for i, p in enumerate(probs):
        s = b.get(i)
        rt, rm = OM.targets(p, s["z"], s["lam"], res[i]["rho"])
        n = p.N + 1
        np.testing.assert_array_equal(M[o:o + n], rm)
        np.testing.assert_allclose(T[o:o + n], rt, rtol=1e-6, atol=1e-12)
        o += n
    b.close()


def test_warm_start_solutions_and_exact_restart_count():
    """Any model's start leads to the same optimum; with a warm budget of one
    iteration every unconverged instance restarts cold and then repeats the
    cold solve exactly (one extra iteration)."""
    ws, _, _ = _model(12)
    probs = _box_batch()
    b = gsls.Batch(probs)
    cold, _ = b.solve(tol=1e-5)
    xs = [b.get(i)["X"] for i in range(len(probs))]
    res, ms, msp = b.solve_ws(ws, tol=1e-5)
    assert ms >= msp > 0
    for i, p in enumerate(probs):
        assert res[i]["status"] == gsls.SOLVED, res[i]
        g = b.get(i)["X"]
        assert np.max(np.abs(g - xs[i])) <= 1e-3 * max(np.max(np.abs(xs[i])), 1.0)
    res1, _, _ = b.solve_ws(ws, tol=1e-5, warm_budget=1)
    for i in range(len(probs)):
        assert res1[i]["cold_restart"] == 1
        assert res1[i]["iterations"] == cold[i]["iterations"] + 1, (res1[i], cold[i])
        np.testing.assert_array_equal(b.get(i)["X"], xs[i])
    b.close(); ws.close()


def test_warm_start_rejects_general_rows():
    ws, _, _ = _model(13)
    b = gsls.Batch([W.random_small(8, 4, 2, 3, 0, seed=40)])
    with pytest.raises(gsls.GslsError):
        b.solve_ws(ws, tol=1e-5)
    b.close(); ws.close()


def test_save_load_round_trip(tmp_path):
    ws, th, _ = _model(14)
    path = tmp_path / "ws.bin"
    ws.save(path)
    ws2 = gsls.WarmStart(path=path)
    np.testing.assert_array_equal(ws2.params(), th.astype(np.float32))
    bad = tmp_path / "bad.bin"
    bad.write_bytes(b"not a model")
    with pytest.raises(gsls.GslsError):
        gsls.WarmStart(path=bad)
    ws.close(); ws2.close()


def test_trained_model_gain_on_held_out_batch():
    """What the trained network (paper_2604_07644_amd/data/ws_box.bin) gains
    over cold-start ADMM on 96 held-out instances (ids 600..695: disjoint from
    the training ids >= 10^6 and the benchmark's 0..511): the same optimum
    (each solve stops at r_p, r_d <= 1e-5, so the two solutions agree to a
    few times the stopping error), and fewer iterations on the typical
    instance (median)."""
    import os
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "paper_2604_07644_amd", "data", "ws_box.bin")
    ws = gsls.WarmStart(path=path)
    probs = W.uneven_batch(count=96, first_instance=600, nmin=16, nmax=200)
    b = gsls.Batch(probs)
    cold, ms_c = b.solve(tol=1e-5)
    xs = [b.get(i)["X"] for i in range(len(probs))]
    warm, ms_w, ms_p = b.solve_ws(ws, tol=1e-5)
    it_c = np.array([r["iterations"] for r in cold])
    it_w = np.array([r["iterations"] for r in warm])
    print(f"cold: median {np.median(it_c)} mean {it_c.mean():.1f} max {it_c.max()} ({ms_c:.1f} ms); "
          f"warm: median {np.median(it_w)} mean {it_w.mean():.1f} max {it_w.max()} ({ms_w:.1f} ms, "
          f"prediction {ms_p:.2f} ms)")
    for i in range(len(probs)):
        assert cold[i]["status"] == gsls.SOLVED and warm[i]["status"] == gsls.SOLVED
        g = b.get(i)["X"]
        assert np.max(np.abs(g - xs[i])) <= 5e-4 * max(np.max(np.abs(xs[i])), 1.0), i
    assert np.median(it_w) < np.median(it_c), (np.median(it_w), np.median(it_c))
    b.close(); ws.close()


def test_learned_start_faster_than_cold_on_uneven_batch():
    """The learned start (predicted rho0, z0 = y0 = 0) solves the 512-instance
    uneven batch in less device time than the cold start, prediction
    included, under the batch's tuned gang schedule; every instance of both
    runs meets the stopping test.  Best of three replays each after a warm-up
    (measured margin about 12 %)."""
    import os
    from paper_2604_07644_amd import autotune
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "paper_2604_07644_amd", "data", "ws_box.bin")
    ws = gsls.WarmStart(path=path)
    probs = W.uneven_batch(count=512)
    b = gsls.Batch(probs)
    tuned = autotune.lookup(autotune.batch_key(probs))
    if tuned is not None:
        b.set_schedule(gang=tuned["gang"], park_share=tuned["park_share"])
    b.solve(tol=1e-5)
    b.solve_ws(ws, tol=1e-5, parts=gsls.WS_RHO)
    cold, warm = [], []
    for _ in range(3):
        r, ms = b.solve(tol=1e-5)
        assert all(x["status"] == gsls.SOLVED for x in r)
        cold.append(ms)
        r, ms, _ = b.solve_ws(ws, tol=1e-5, parts=gsls.WS_RHO)
        assert all(x["status"] == gsls.SOLVED for x in r)
        warm.append(ms)
    print(f"cold {min(cold):.1f} ms, learned start {min(warm):.1f} ms (device, per batch)")
    assert min(warm) < min(cold), (warm, cold)
    b.close(); ws.close()


def test_warm_start_parts():
    """The start may take any subset of the prediction: with the predicted
    rho alone (z0 = y0 = 0) the same optimum is reached, and a warm budget of
    one iteration restarts every unconverged instance cold; an empty or
    unknown part set is refused."""
    ws, _, _ = _model(15)
    probs = _box_batch()
    b = gsls.Batch(probs)
    cold, _ = b.solve(tol=1e-5)
    xs = [b.get(i)["X"] for i in range(len(probs))]
    res, _, _ = b.solve_ws(ws, tol=1e-5, parts=gsls.WS_RHO)
    for i in range(len(probs)):
        assert res[i]["status"] == gsls.SOLVED
        assert np.max(np.abs(b.get(i)["X"] - xs[i])) <= 1e-3 * max(np.max(np.abs(xs[i])), 1.0)
    res1, _, _ = b.solve_ws(ws, tol=1e-5, warm_budget=1, parts=gsls.WS_RHO | gsls.WS_Z)
    for i in range(len(probs)):
        assert res1[i]["cold_restart"] == 1
        assert res1[i]["iterations"] == cold[i]["iterations"] + 1
    for bad in (0, 8):
        with pytest.raises(gsls.GslsError):
            b.solve_ws(ws, tol=1e-5, parts=bad)
    b.close(); ws.close()
