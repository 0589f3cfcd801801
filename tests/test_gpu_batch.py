"""GPU parity of the batched submit path (persistent per-pass launches over
uneven shapes, graph capture and replay, autotuner) against the FP64 oracle,
through the C ABI.

Tolerance: relative L2 <= 1e-6 per array (the maximum over the batch is
reported in the assertion).  A batched item computes each row and column
exactly as it would alone, so an item's result alone and inside a mix must be
bitwise equal."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL = 1e-6


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2110_01172_amd as dx
    from paper_2110_01172_amd import inputs
    import oracle
    oracle.build(force=False)
    return torch, dx, inputs, oracle


def _ref(oracle, kind, x, norm="backward", hh=(0.0, 0.0)):
    if kind in ("dct2d", "dct3d"):
        return oracle.dctn(x, norm)
    if kind in ("idct2d", "idct3d"):
        return oracle.idctn(x, norm)
    n1, n2 = x.shape
    return oracle.poisson2d_neumann(x, hh[0] if hh[0] > 0 else None, hh[1] if hh[1] > 0 else None)


def _make(env, specs, seed):
    torch, _, inputs, _ = env
    items, xs = [], []
    for i, (kind, shape, norm, hh) in enumerate(specs):
        x = inputs.uniform(shape, seed + i)
        xs.append(x)
        xt = torch.from_numpy(x).cuda()
        items.append((kind, xt, torch.full_like(xt, float("nan")), norm, hh))
    return items, xs


def _check(env, specs, items, xs, idx=None):
    _, _, _, oracle = env
    worst = 0.0
    for i in (range(len(specs)) if idx is None else idx):
        kind, _, norm, hh = specs[i]
        y = items[i][2].cpu().numpy()
        err = oracle.rel_l2(y, _ref(oracle, kind, xs[i], norm, hh))
        worst = max(worst, err)
        assert err <= TOL, f"item {i} {kind} {xs[i].shape} {norm}: rel L2 {err:.3e}"
    return worst


def test_uneven_dct2_batch_64(env):
    torch, dx, inputs, _ = env
    shapes = inputs.uneven_batch_shapes(64, 3000)
    specs = [("dct2d", s, "backward", None) for s in shapes]
    items, xs = _make(env, specs, 3100)
    print(f"[gpu] submit_batch 64 uneven dct2d", flush=True)
    dx.submit_batch(items)
    torch.cuda.synchronize()
    _check(env, specs, items, xs)


def test_shuffled_tile_order_is_bitwise_identical(env):
    """The persistent batch passes walk their tiles in any order with the same
    result: a mixed batch (DCT, IDCT, Poisson; uneven shapes, odd ones
    included) submitted with the normal largest-first order and with two
    seeded random tile orders (DCTX_BATCH_SHUFFLE) is bitwise the same, and
    matches the oracle."""
    import os
    torch, dx, inputs, _ = env
    shapes = inputs.uneven_batch_shapes(40, 3970) + [(45, 75), (64, 9), (250, 486)]
    kinds = ["dct2d", "idct2d", "poisson2d"]
    specs = [(kinds[i % 3], s, "backward" if i % 2 else "ortho", None) for i, s in enumerate(shapes)]
    specs = [(k, s, None, (0.0, 0.0)) if k == "poisson2d" else (k, s, n, h) for k, s, n, h in specs]
    items, xs = _make(env, specs, 3980)
    print("[gpu] batch tile-order shuffle", flush=True)
    dx.submit_batch(items)
    torch.cuda.synchronize()
    base = [it[2].clone() for it in items]
    for seed in ("7", "12345"):
        for it in items:
            it[2].fill_(float("nan"))
        os.environ["DCTX_BATCH_SHUFFLE"] = seed
        try:
            dx.submit_batch(items)
            torch.cuda.synchronize()
        finally:
            del os.environ["DCTX_BATCH_SHUFFLE"]
        for i, it in enumerate(items):
            assert torch.equal(it[2], base[i]), f"seed {seed}: item {i} {specs[i][:2]} differs"
    _check(env, specs, items, xs)


def test_batch_object_resubmits(env):
    """A Batch built once and submitted twice writes the same outputs, equal to
    the oracle (the descriptor array is reused, the tensors kept alive)."""
    torch, dx, inputs, _ = env
    shapes = inputs.uneven_batch_shapes(24, 3050)
    specs = [("dct2d", s, "backward", None) for s in shapes]
    items, xs = _make(env, specs, 3150)
    b = dx.Batch(items)
    print(f"[gpu] Batch resubmit 24 uneven dct2d", flush=True)
    b.submit()
    torch.cuda.synchronize()
    first = [it[2].clone() for it in items]
    for it in items:
        it[2].fill_(float("nan"))
    b.submit()
    torch.cuda.synchronize()
    for a, it in zip(first, items):
        assert torch.equal(a, it[2])
    _check(env, specs, items, xs)


def test_mixed_kinds_batch(env):
    torch, dx, _, _ = env
    specs = [("dct2d", (64, 100), "ortho", None), ("idct2d", (90, 48), "backward", None),
             ("poisson2d", (128, 96), None, (0.0, 0.0)), ("dct3d", (12, 10, 16), "backward", None),
             ("idct3d", (8, 6, 20), "ortho", None), ("dct2d", (1000, 64), "backward", None),
             ("idct2d", (6, 10), "ortho", None), ("poisson2d", (30, 40), None, (0.5, 0.25)),
             ("dct2d", (256, 256), "backward", None), ("idct2d", (512, 1024), "backward", None)]
    items, xs = _make(env, specs, 3200)
    print(f"[gpu] submit_batch mixed kinds", flush=True)
    dx.submit_batch(items)
    torch.cuda.synchronize()
    _check(env, specs, items, xs)


def test_alone_equals_in_mix(env):
    torch, dx, inputs, _ = env
    shapes = inputs.uneven_batch_shapes(24, 3300)
    specs = [(("dct2d", "idct2d", "poisson2d")[i % 3], s, "backward", (0.0, 0.0)) for i, s in enumerate(shapes)]
    items, xs = _make(env, specs, 3400)
    print(f"[gpu] alone vs mix", flush=True)
    dx.submit_batch(items)
    torch.cuda.synchronize()
    for i in (0, 5, 13, 23):
        kind, xt, out = items[i][0], items[i][1], items[i][2]
        alone = torch.full_like(xt, float("nan"))
        dx.submit_batch([(kind, xt, alone, "backward", (0.0, 0.0))])
        torch.cuda.synchronize()
        assert torch.equal(alone, out), f"item {i} differs alone vs in the mix"


def test_config3_batch_512_sampled(env):
    """512 arrays, sides uniform over the 50 even 5-smooth sizes in [64, 1024],
    uniform[-1, 1]: 32 random arrays against the oracle."""
    torch, dx, inputs, _ = env
    shapes = inputs.uneven_batch_shapes(512, 3000)
    specs = [("dct2d", s, "backward", None) for s in shapes]
    items, xs = _make(env, specs, 3500)
    print(f"[gpu] submit_batch 512 (config 3)", flush=True)
    dx.submit_batch(items)
    torch.cuda.synchronize()
    idx = sorted(np.random.default_rng(3).choice(512, 32, replace=False).tolist())
    _check(env, specs, items, xs, idx)
    for i in range(512):
        assert bool(torch.isfinite(items[i][2]).all()), f"item {i} not fully written"


def test_graph_replays(env):
    """Captured batch replayed three times with eager work in between; every
    replay equals the eager submit."""
    torch, dx, inputs, _ = env
    shapes = inputs.uneven_batch_shapes(16, 3600)
    specs = [(("dct2d", "idct2d", "poisson2d")[i % 3], s, "backward", (0.0, 0.0)) for i, s in enumerate(shapes)]
    specs.append(("dct3d", (16, 12, 10), "backward", None))
    items, xs = _make(env, specs, 3700)
    dx.submit_batch(items)
    torch.cuda.synchronize()
    eager = [it[2].clone() for it in items]
    print(f"[gpu] graph create + 3 replays", flush=True)
    g = dx.BatchGraph(items)
    try:
        for rep in range(3):
            for it in items:
                it[2].zero_()
            junk = torch.randn(1 << 20, device="cuda")
            junk.mul_(2.0).sum().item()
            g.launch()
            torch.cuda.synchronize()
            for i, it in enumerate(items):
                assert torch.equal(it[2], eager[i]), f"replay {rep} item {i} differs"
    finally:
        g.close()
    _check(env, specs, items, xs)


def test_autotune_then_submit(env):
    torch, dx, inputs, _ = env
    shapes = inputs.uneven_batch_shapes(48, 3800)
    specs = [("dct2d", s, "backward", None) for s in shapes]
    items, xs = _make(env, specs, 3900)
    print(f"[gpu] autotune 48", flush=True)
    info = dx.autotune_batch(items)
    assert info["tuned_ms"] > 0 and info["tuned_ms"] <= info["default_ms"] * 1.5
    assert set(info["passes"]) == {"dct_rows", "dct_cols"}
    for it in items:
        it[2].fill_(float("nan"))
    dx.submit_batch(items)
    torch.cuda.synchronize()
    _check(env, specs, items, xs)


def test_tune_cache_file_round_trip(env, tmp_path):
    """The autotuner's choices written to a JSON file (keyed by gfx arch and
    batch signature) and loaded into a fresh handle give that handle the same
    launch geometry: the batch then runs bitwise the same as on the tuned
    handle, and the oracle check holds."""
    import json
    torch, dx, inputs, _ = env
    shapes = inputs.uneven_batch_shapes(24, 3950)
    specs = [("dct2d", s, "backward", None) for s in shapes]
    items, xs = _make(env, specs, 3960)
    tuned = dx.Handle(0)
    print("[gpu] autotune 24 + cache file", flush=True)
    info = dx.autotune_batch(items, handle=tuned)
    path = str(tmp_path / "tune.json")
    dx.tune_save(path, handle=tuned)
    doc = json.load(open(path))
    assert doc["format"] == "dctx-tune-1" and len(doc["entries"]) >= 1
    e = doc["entries"][0]
    assert e["arch"].startswith("gfx") and len(e["signature"]) == 16
    assert e["per_cap"][0] == info["passes"]["dct_rows"]["per_cap"]
    fresh = dx.Handle(0)
    assert dx.tune_load(path, handle=fresh) == len(doc["entries"])
    dx.submit_batch(items, handle=tuned)
    first = [it[2].clone() for it in items]
    for it in items:
        it[2].fill_(float("nan"))
    dx.submit_batch(items, handle=fresh)
    torch.cuda.synchronize()
    for a, it in zip(first, items):
        assert torch.equal(a, it[2])
    _check(env, specs, items, xs)
    with pytest.raises(dx.DctxError):
        dx.tune_load(str(tmp_path / "missing.json"), handle=fresh)


def test_batch_rejects_and_enqueues_nothing(env):
    torch, dx, _, _ = env
    a = torch.zeros((64, 64), device="cuda")
    b = torch.full((64, 64), 7.0, device="cuda")
    c = torch.zeros((64, 64), device="cuda")
    # two items writing the same output
    with pytest.raises(dx.DctxError):
        dx.submit_batch([("dct2d", a, b), ("dct2d", c, b)])
    # one unsupported item (last dimension not 5-smooth) among good ones
    d = torch.zeros((8, 7), device="cuda")
    e = torch.full((8, 7), 7.0, device="cuda")
    with pytest.raises(dx.DctxError) as ei:
        dx.submit_batch([("dct2d", a, b), ("dct2d", d, e)])
    assert "ERR_UNSUPPORTED" in str(ei.value)
    torch.cuda.synchronize()
    assert bool((b == 7.0).all()) and bool((e == 7.0).all())


def test_batch_odd_and_two_last_dimension(env):
    """Items with an odd contiguous dimension (full-length row FFTs, column 0
    alone) and with n2 = 2 (a length-1 row FFT) in one batch with even ones,
    every kind: each against the oracle, and bitwise equal to the same item
    submitted alone."""
    torch, dx, _, _ = env
    specs = [("dct2d", (9, 15), "backward", None), ("idct2d", (64, 75), "ortho", None),
             ("poisson2d", (100, 81), "backward", (0.0, 0.0)), ("dct2d", (250, 45), "ortho", None),
             ("idct2d", (48, 2), "backward", None), ("poisson2d", (64, 2), "backward", (0.0, 0.0)),
             ("dct2d", (96, 128), "backward", None), ("idct2d", (27, 125), "backward", None),
             ("dct2d", (512, 375), "backward", None), ("poisson2d", (30, 25), "backward", (0.1, 0.2))]
    items, xs = _make(env, specs, 3700)
    print("[gpu] submit_batch odd / two last dimension", flush=True)
    dx.submit_batch(items)
    torch.cuda.synchronize()
    _check(env, specs, items, xs)
    for i in (0, 2, 4, 7):
        kind, xt, out, norm, hh = items[i]
        alone = torch.full_like(xt, float("nan"))
        dx.submit_batch([(kind, xt, alone, norm, hh)])
        torch.cuda.synchronize()
        assert torch.equal(alone, out), f"item {i} {kind} {tuple(xt.shape)} differs alone vs in the mix"
