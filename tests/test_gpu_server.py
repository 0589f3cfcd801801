"""GPU tests of the continuous-batching serving loop through the C ABI:
results equal the oracle (FP32 tolerance) and are bitwise the same alone and
in a mix; admission respects the HBM budget and the arrival times; the
per-request (plain) mode serves the same requests."""
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


def _ref(oracle, kind, x):
    if kind in ("dct2d", "dct3d"):
        return oracle.dctn(x)
    if kind in ("idct2d", "idct3d"):
        return oracle.idctn(x)
    return oracle.poisson2d_neumann(x)


SPECS = [("dct2d", (64, 64)), ("idct2d", (128, 96)), ("poisson2d", (96, 128)), ("dct3d", (16, 16, 16)),
         ("dct2d", (256, 250)), ("idct3d", (8, 12, 20)), ("poisson2d", (64, 64)), ("dct2d", (1000, 64)),
         ("idct2d", (30, 40)), ("dct2d", (512, 512)), ("dct3d", (32, 24, 40)), ("poisson2d", (250, 486))]


def _make(env, seed, reps=1):
    torch, _, inputs, _ = env
    items, xs = [], []
    for r in range(reps):
        for i, (kind, shape) in enumerate(SPECS):
            x = inputs.uniform(shape, seed + 100 * r + i)
            xt = torch.from_numpy(x).cuda()
            items.append((kind, xt, torch.full_like(xt, float("nan"))))
            xs.append(x)
    return items, xs


def test_server_mix_matches_oracle_and_alone(env):
    torch, dx, _, oracle = env
    items, xs = _make(env, 6000, reps=3)
    print("[gpu] server mix of 36 requests", flush=True)
    srv = dx.Server(hbm_budget=256 << 20, max_inflight=64, nstreams=4)
    try:
        t0 = srv.now()
        tickets = [srv.submit(it, t0 + 0.0002 * k) for k, it in enumerate(items)]
        srv.drain()
        stats = [srv.poll(t) for t in tickets]
        assert all(s is not None and s["status"] == "OK" for s in stats)
        assert all(s["launch_s"] >= s["arrival_s"] for s in stats)
        assert max(s["batch_size"] for s in stats) >= 1
        for k, (kind, xt, out) in enumerate(items):
            err = oracle.rel_l2(out.cpu().numpy(), _ref(oracle, kind, xs[k]))
            assert err <= TOL, f"request {k} {kind} {tuple(xt.shape)}: rel L2 {err:.3e}"
        # the same requests alone (one at a time) give bitwise the same results
        for k in (0, 2, 3, 7, 11, 20, 35):
            kind, xt, out = items[k]
            alone = torch.full_like(xt, float("nan"))
            tk = srv.submit((kind, xt, alone))
            srv.drain()
            assert srv.poll(tk)["batch_size"] == 1
            assert torch.equal(alone, out), f"request {k} differs alone vs in the mix"
        sm = srv.summary()
        assert sm["completed"] == len(items) + 7 and sm["p99_ms"] >= sm["p50_ms"] > 0
        assert sm["peak_pool_bytes"] <= 256 << 20
    finally:
        srv.close()


def test_server_small_budget_queues(env):
    """A pool that holds only one large request at a time: everything still
    completes, in FIFO order of admission, within the budget."""
    torch, dx, _, oracle = env
    items, xs = _make(env, 6100)
    budget = 1 << 20   # the 512^2 DCT needs 512 * 256 * 8 = 1 MiB
    print("[gpu] server with a 1 MiB pool", flush=True)
    srv = dx.Server(hbm_budget=budget, max_inflight=8, nstreams=2)
    try:
        tickets = [srv.submit(it) for it in items]
        srv.drain()
        for k, tk in enumerate(tickets):
            st = srv.poll(tk)
            assert st["status"] == "OK"
            kind, xt, out = items[k]
            assert oracle.rel_l2(out.cpu().numpy(), _ref(oracle, kind, xs[k])) <= TOL
        assert srv.summary()["peak_pool_bytes"] <= budget
        big = torch.zeros((1024, 1024), device="cuda")
        with pytest.raises(dx.DctxError):
            srv.submit(("dct2d", big, torch.empty_like(big)))   # 4 MiB workspace > pool
    finally:
        srv.close()


def test_server_plain_mode(env):
    torch, dx, _, oracle = env
    items, xs = _make(env, 6200)
    print("[gpu] plain-mode server", flush=True)
    srv = dx.Server(plain=True, max_inflight=4)
    try:
        tickets = [srv.submit(it) for it in items]
        srv.drain()
        for k, tk in enumerate(tickets):
            assert srv.poll(tk)["batch_size"] == 1
            kind, xt, out = items[k]
            assert oracle.rel_l2(out.cpu().numpy(), _ref(oracle, kind, xs[k])) <= TOL
    finally:
        srv.close()


def test_server_rejects_bad_request(env):
    torch, dx, _, _ = env
    srv = dx.Server(hbm_budget=16 << 20)
    try:
        a = torch.zeros((8, 7), device="cuda")
        with pytest.raises(dx.DctxError):
            srv.submit(("dct2d", a, torch.empty_like(a)))
        b = torch.zeros((8, 8), device="cuda")
        with pytest.raises(dx.DctxError):
            srv.submit(("dct2d", b, b))   # in place
    finally:
        srv.close()
