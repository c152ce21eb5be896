"""GPU surrogate network against its FP64 NumPy reference: forward pass,
gradients (per tensor, relative 2-norm), and a short training run.
Bars: FP32 products 1e-4, BF16 products 2e-2."""
import numpy as np
import pytest

from oracle import surrogate_ref as sr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1310_6380_amd import mvpb
    c = mvpb.Context(0)
    yield c
    c.close()


def _batch(B, seed):
    rng = np.random.default_rng(seed)
    cells = (rng.uniform(size=(B, 32, 32)) > 0.5).astype(np.uint8)
    target = rng.uniform(0.2, 1.5, (B, sr.N_OUT)).astype(np.float32)
    return cells, target


def _nudge_biases(theta, rng):
    o = 0
    for s in sr.param_shapes():
        n = int(np.prod(s))
        if len(s) == 1:
            theta[o:o + n] = rng.uniform(-0.2, 0.2, n)
        o += n
    return theta


@pytest.mark.parametrize("prec,tol", [(0, 1e-4), (1, 2e-2)])
def test_forward_matches_reference(ctx, prec, tol):
    from paper_1310_6380_amd import mvpb
    print("surrogate forward", prec, flush=True)
    net = mvpb.Surrogate(ctx, max_batch=16, precision=prec, seed=11)
    theta = _nudge_biases(net.get_params().astype(np.float64), np.random.default_rng(0))
    net.set_params(theta)
    theta = net.get_params().astype(np.float64)          # exactly the FP32 values the GPU holds
    cells, _ = _batch(16, 1)
    out = net.infer(cells)
    ref = sr.forward(theta, cells.astype(np.float64))
    err = np.linalg.norm(out - ref) / np.linalg.norm(ref)
    print("  rel err", err, flush=True)
    assert err <= tol
    net.close()


@pytest.mark.parametrize("prec,tol", [(0, 1e-4), (1, 2e-2)])
def test_gradients_match_reference(ctx, prec, tol):
    from paper_1310_6380_amd import mvpb
    print("surrogate gradients", prec, flush=True)
    net = mvpb.Surrogate(ctx, max_batch=8, precision=prec, seed=5)
    theta = _nudge_biases(net.get_params().astype(np.float64), np.random.default_rng(2))
    net.set_params(theta)
    theta = net.get_params().astype(np.float64)
    cells, target = _batch(8, 3)
    loss, g = net.gradients(cells, target)
    L, gref = sr.gradients(theta, cells.astype(np.float64), target.astype(np.float64))
    assert abs(loss - L) <= tol * L
    o = 0
    for s in sr.param_shapes():
        n = int(np.prod(s))
        a, b = g[o:o + n], gref[o:o + n]
        err = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        print("  tensor", s, "rel err", err, flush=True)
        assert err <= tol, (s, err)
        o += n
    net.close()


def test_training_reduces_loss(ctx):
    from paper_1310_6380_amd import mvpb
    net = mvpb.Surrogate(ctx, max_batch=32, precision=1, seed=7)
    cells, target = _batch(32, 9)
    first = net.train_step(cells, target, 1e-3)
    for _ in range(40):
        last = net.train_step(cells, target, 1e-3)
    print("loss", first, "->", last, flush=True)
    assert last < 0.5 * first
    net.close()


def test_labels_training_and_screening(ctx):
    """The workflow on a small scale: labels from the batched solver (checked
    against the oracle), training on shifted batches, held-out error, and one
    screening round whose top candidates are verified by the plain solve."""
    from oracle import mixed_oracle as mo
    from oracle.compare import band_error
    from paper_1310_6380_amd import mvpb, screening as sc
    from synth import config4_cells, kpath_gxmg

    cells = config4_cells(0, 96)
    print("labels", flush=True)
    y = sc.label_cells(ctx, cells)
    assert y.shape == (96, 400) and np.all(np.isfinite(y))
    Q = kpath_gxmg(40)
    props = np.array([sc.MATRIX, sc.INCLUSION])
    for i in (0, 1):
        ref, _ = mo.bands(cells[i].astype(np.int32), props, np.eye(2), 7, 7, Q[[0, 15, 30]], 10)
        got = y[i].reshape(40, 10)[[0, 15, 30]].astype(np.float64) * 2 * np.pi * sc.C_REF
        # labels are stored as float32 (the solve itself is FP64)
        assert band_error(got, ref) <= 1e-6
    net = mvpb.Surrogate(ctx, max_batch=4096, precision=1, seed=1)
    losses = sc.train(net, cells[:64], y[:64], epochs=10, batch=32, lr=2e-3)
    assert losses[-1] < losses[0]
    err = sc.relative_errors(net.infer(cells[64:]), y[64:])
    print("held-out median rel err", float(np.median(err)), flush=True)
    assert np.all(np.isfinite(err))
    stats = sc.screen(ctx, net, cells[:16], b=2, rounds=1, n_candidates=512, top_k=4)
    assert stats["verified"] == 4 and 0 <= stats["fallbacks"] <= 4
    per_pred = stats["t_surrogate"] / stats["predicted"]
    per_solve = stats["t_solve"] / stats["verified"]
    print("surrogate s/cell", per_pred, "solve s/cell", per_solve, flush=True)
    assert per_solve > 10 * per_pred
    net.close()


def test_screening_fallback_with_zero_tolerance(ctx):
    """A zero tolerance sends every verified candidate to the plain solve."""
    from paper_1310_6380_amd import mvpb, screening as sc
    from synth import config4_cells
    cells = config4_cells(100, 116)
    net = mvpb.Surrogate(ctx, max_batch=256, precision=1, seed=2)
    stats = sc.screen(ctx, net, cells, b=2, rounds=1, n_candidates=64, top_k=3, tol=0.0)
    assert stats["fallbacks"] == stats["verified"] == 3
    net.close()


def test_checkpoint_resumes_training_exactly(ctx, tmp_path):
    """Save after a few Adam steps, load into a new network: the parameters
    are equal, and the next steps of both networks give identical losses and
    parameters (the moments and the step counter were restored)."""
    from paper_1310_6380_amd import mvpb
    print("surrogate checkpoint", flush=True)
    net = mvpb.Surrogate(ctx, max_batch=8, precision=1, seed=3)
    cells, target = _batch(8, 4)
    for _ in range(3):
        net.train_step(cells, target, 1e-3)
    path = str(tmp_path / "sur.ckpt")
    net.save(path)
    net2 = mvpb.Surrogate.load(ctx, path, max_batch=8)
    assert np.array_equal(net.get_params(), net2.get_params())
    after = []
    for _ in range(2):
        assert net.train_step(cells, target, 1e-3) == net2.train_step(cells, target, 1e-3)
        after.append(net.get_params())
    assert np.array_equal(net.get_params(), net2.get_params())
    # the same parameters with the moments cleared take a different step
    net3 = mvpb.Surrogate(ctx, max_batch=8, precision=1, seed=3)
    net3.set_params(mvpb.Surrogate.load(ctx, path, max_batch=8).get_params())
    net3.train_step(cells, target, 1e-3)
    assert not np.array_equal(net3.get_params(), after[0])
    bad = tmp_path / "bad.ckpt"
    bad.write_bytes(b"not a checkpoint")
    with pytest.raises(mvpb.MvpbError) as ei:
        mvpb.Surrogate.load(ctx, str(bad))
    assert ei.value.code == mvpb.E_INVALID
    for n in (net, net2, net3):
        n.close()


def test_surrogate_ranking_beats_random_selection(ctx):
    """What the trained network gains over the method without it: with the
    same budget of plain solves (32 cells verified), the candidates the
    surrogate ranks highest by predicted gap hold a larger verified gap than
    randomly chosen candidates.  Trained on 8192 seeded GRF cells, candidates
    are 1024 cells it has not seen, their bands (the verification) computed by
    the batched FP64 solver."""
    from paper_1310_6380_amd import mvpb, screening as sc
    from synth import config4_cells
    cells = config4_cells(0, 9216)
    print("labels", flush=True)
    y = sc.label_cells(ctx, cells)
    train, pool = slice(0, 8192), slice(8192, 9216)
    norm = sc.Normalizer(y[train])
    net = mvpb.Surrogate(ctx, max_batch=4096, precision=1, seed=3)
    sc.train(net, cells[train], y[train], epochs=60, batch=256, lr=2e-3, lr_end=2e-5, norm=norm)
    pred = sc.predict(net, cells[pool], norm)
    net.close()
    b, budget = 2, 32
    true_gap = sc.band_gap(y[pool], b)
    pick = np.argsort(-sc.band_gap(pred, b))[:budget]
    best_s, mean_s = true_gap[pick].max(), true_gap[pick].mean()
    rng = np.random.default_rng(0)
    draws = np.stack([rng.choice(true_gap.size, budget, replace=False) for _ in range(400)])
    best_r, mean_r = true_gap[draws].max(axis=1), true_gap[draws].mean(axis=1)
    frac = float(np.mean(true_gap >= best_s))
    print(f"surrogate: best {best_s:.4f} mean {mean_s:.4f}; random: best p50 {np.median(best_r):.4f} "
          f"p90 {np.percentile(best_r, 90):.4f} mean {mean_r.mean():.4f}; "
          f"random solves to reach the surrogate's best ~ {1.0 / max(frac, 1e-9):.0f}", flush=True)
    assert best_s >= np.percentile(best_r, 90)
    assert mean_s > np.percentile(mean_r, 99)
