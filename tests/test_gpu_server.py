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
         ("idct2d", (30, 40)), ("dct2d", (512, 512)), ("dct3d", (32, 24, 40)), ("poisson2d", (250, 486)),
         ("dct2d", (50, 45)), ("poisson2d", (30, 25)), ("idct2d", (40, 2))]

# requests of the compile-time kernels (run as grouped launches inside a
# batch): a 2^20-element 2-D DCT and IDCT, a 2048^2 DCT (split form), 3-D
# DCT / IDCT at 64^3, and Poisson solves at 256^2 and 1024^2
BIG = [("dct2d", (1024, 1024)), ("idct2d", (1024, 1024)), ("dct2d", (2048, 2048)), ("dct3d", (64, 64, 64)),
       ("idct3d", (64, 64, 64)), ("poisson2d", (256, 256)), ("poisson2d", (1024, 1024)), ("dct2d", (256, 256))]


def _make(env, seed, reps=1, specs=SPECS):
    torch, _, inputs, _ = env
    items, xs = [], []
    for r in range(reps):
        for i, (kind, shape) in enumerate(specs):
            x = inputs.uniform(shape, seed + 100 * r + i)
            xt = torch.from_numpy(x).cuda()
            items.append((kind, xt, torch.full_like(xt, float("nan"))))
            xs.append(x)
    return items, xs


def _check_alone(torch, srv, items, picks):
    """Each picked request submitted alone (a batch of one) gives bitwise the
    result it had in the mix."""
    for k in picks:
        kind, xt, out = items[k]
        alone = torch.full_like(xt, float("nan"))
        tk = srv.submit((kind, xt, alone))
        srv.drain()
        assert srv.poll(tk)["batch_size"] == 1
        assert torch.equal(alone, out), f"request {k} {kind} {tuple(xt.shape)} differs alone vs in the mix"


def test_server_batch_matches_oracle_and_alone(env):
    """One burst: every request arrives at the same instant, so the scheduler
    admits them as one batch (small ones in the persistent batch passes,
    same-shape power-of-two ones as grouped launches).  Every result matches
    the oracle, every request ran in a batch of more than one, and each is
    bitwise the same when run alone."""
    torch, dx, _, oracle = env
    items, xs = _make(env, 6000, reps=1)
    big, xb = _make(env, 6050, reps=2, specs=BIG)
    items += big
    xs += xb
    print(f"[gpu] server burst of {len(items)} requests", flush=True)
    srv = dx.Server(hbm_budget=1 << 30, max_inflight=64, nstreams=4, max_batch=64)
    try:
        # plans and kernels built beforehand, so the burst is one scheduler pass
        for it in items:
            srv.submit((it[0], it[1], torch.empty_like(it[1])))
        srv.drain()
        t0 = srv.now() + 0.02
        tickets = [srv.submit(it, t0) for it in items]
        srv.drain()
        stats = [srv.poll(t) for t in tickets]
        sizes = [s["batch_size"] for s in stats]
        print(f"[gpu] burst batch sizes: {sorted(set(sizes))}", flush=True)
        assert all(s is not None and s["status"] == "OK" for s in stats)
        assert all(s["launch_s"] >= s["arrival_s"] for s in stats)
        assert min(sizes) > 1, f"a request of the burst ran alone: {sizes}"
        for k, (kind, xt, out) in enumerate(items):
            err = oracle.rel_l2(out.cpu().numpy(), _ref(oracle, kind, xs[k]))
            assert err <= TOL, f"request {k} {kind} {tuple(xt.shape)}: rel L2 {err:.3e}"
        # every BIG shape twice in the burst: both copies of a shape ran as one
        # grouped launch; all of them, and small ones, alone
        _check_alone(torch, srv, items, [0, 2, 3, 7, 11] + list(range(len(SPECS), len(items))))
    finally:
        srv.close()


def test_server_continuous_admission(env):
    """Arrivals spaced closer than the service time behind a long head batch:
    requests arriving while batches run are gathered into batches of more than
    one, a batch is launched while an earlier one is still on the GPU, and
    every result matches the oracle and its alone run bitwise."""
    torch, dx, _, oracle = env
    head, xh = _make(env, 6080, reps=4, specs=[("dct2d", (2048, 2048))])
    tail, xt_ = _make(env, 6090, reps=2, specs=SPECS + BIG)
    items, xs = head + tail, xh + xt_
    print(f"[gpu] server stream of {len(items)} requests", flush=True)
    srv = dx.Server(hbm_budget=2 << 30, max_inflight=64, nstreams=4, max_batch=16, min_batch=4)
    try:
        for it in items:
            srv.submit((it[0], it[1], torch.empty_like(it[1])))
        srv.drain()
        t0 = srv.now() + 0.02
        arr = [t0] * len(head) + [t0 + 2e-5 + 5e-6 * k for k in range(len(tail))]
        tickets = [srv.submit(it, a) for it, a in zip(items, arr)]
        srv.drain()
        stats = [srv.poll(t) for t in tickets]
        assert all(s["status"] == "OK" for s in stats)
        sizes = [s["batch_size"] for s in stats]
        print(f"[gpu] stream batch sizes: {sizes}", flush=True)
        assert max(sizes[len(head):]) > 1, "no arrivals were gathered into a batch"
        # some batch launched while another (launched earlier) had not completed
        spans = sorted({(s["launch_s"], s["done_s"]) for s in stats})
        assert any(spans[j][0] < spans[i][1] for i in range(len(spans)) for j in range(i + 1, len(spans))), \
            "no batch overlapped another on the GPU"
        for k, (kind, xt, out) in enumerate(items):
            err = oracle.rel_l2(out.cpu().numpy(), _ref(oracle, kind, xs[k]))
            assert err <= TOL, f"request {k} {kind} {tuple(xt.shape)}: rel L2 {err:.3e}"
        _check_alone(torch, srv, items, [0, len(head), len(head) + 3, len(head) + len(SPECS) + 2, len(items) - 1])
        sm = srv.summary()
        assert sm["p99_ms"] >= sm["p50_ms"] > 0
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


def test_server_cancel(env):
    """Requests cancelled before launch complete as cancelled and their
    buffers are never touched; the others complete normally and match the
    oracle.  Cancelling a done request reports False; an unknown ticket is an
    error.  A cancel racing the scheduler either wins (cancelled, untouched)
    or loses (normal completion)."""
    torch, dx, _, oracle = env
    items, xs = _make(env, 6300)
    for _, _, out in items:
        out.fill_(7.0)
    print(f"[gpu] server cancel over {len(items)} requests", flush=True)
    srv = dx.Server(hbm_budget=1 << 30, max_inflight=64, nstreams=2, max_batch=8)
    try:
        t0 = srv.now() + 0.5   # far enough ahead that nothing arrives before the cancels
        tickets = [srv.submit(it, t0) for it in items]
        gone = set(range(0, len(items), 2))
        for k in gone:
            assert srv.cancel(tickets[k])
        srv.drain()
        for k, tk in enumerate(tickets):
            st = srv.poll(tk)
            kind, xt, out = items[k]
            if k in gone:
                assert st["status"] == "ERR_CANCELLED" and st["batch_size"] == 0
                assert bool((out == 7.0).all()), f"cancelled request {k} touched its output"
            else:
                assert st["status"] == "OK"
                assert oracle.rel_l2(out.cpu().numpy(), _ref(oracle, kind, xs[k])) <= TOL
        assert not srv.cancel(tickets[1])   # done
        with pytest.raises(dx.DctxError):
            srv.cancel(10 ** 9)
        assert srv.summary(tickets[0])["completed"] == len(items) - len(gone)
        # racing cancels of requests that arrive at once
        items2, xs2 = _make(env, 6400)
        for _, _, out in items2:
            out.fill_(7.0)
        tk2 = [srv.submit(it) for it in items2]
        won = [srv.cancel(t) for t in tk2[::-1]][::-1]
        srv.drain()
        for k, tk in enumerate(tk2):
            st = srv.poll(tk)
            kind, xt, out = items2[k]
            if won[k]:
                assert st["status"] == "ERR_CANCELLED" and bool((out == 7.0).all())
            else:
                assert st["status"] == "OK"
                assert oracle.rel_l2(out.cpu().numpy(), _ref(oracle, kind, xs2[k])) <= TOL
        print(f"[gpu] racing cancels won {sum(won)} of {len(won)}", flush=True)
    finally:
        srv.close()


@pytest.mark.parametrize("plain", [False, True])
def test_server_injected_alloc_failure(env, plain):
    """Injected allocation failures: the affected batches' requests complete
    with ERR_NOMEM and untouched outputs, every other request completes and
    matches the oracle, the pool and slots are released (a later wave runs
    in full), and the summary counts successes only."""
    torch, dx, _, oracle = env
    items, xs = _make(env, 6500)
    for _, _, out in items:
        out.fill_(7.0)
    print(f"[gpu] server injected failures plain={plain}", flush=True)
    srv = dx.Server(hbm_budget=1 << 30, max_inflight=64, nstreams=2, max_batch=4, plain=plain)
    try:
        srv.inject_alloc_failures(2)
        t0 = srv.now() + 0.05
        tickets = [srv.submit(it, t0) for it in items]
        srv.drain()
        stats = [srv.poll(t) for t in tickets]
        failed = [k for k, s in enumerate(stats) if s["status"] != "OK"]
        assert failed and all(stats[k]["status"] == "ERR_NOMEM" for k in failed)
        assert len(failed) <= (2 if plain else 8)
        for k, (kind, xt, out) in enumerate(items):
            if k in failed:
                assert bool((out == 7.0).all()), f"failed request {k} touched its output"
            else:
                assert oracle.rel_l2(out.cpu().numpy(), _ref(oracle, kind, xs[k])) <= TOL
        assert srv.summary(tickets[0])["completed"] == len(items) - len(failed)
        # serving goes on: a second wave completes in full
        items2, xs2 = _make(env, 6600)
        tk2 = [srv.submit(it) for it in items2]
        srv.drain()
        for k, tk in enumerate(tk2):
            assert srv.poll(tk)["status"] == "OK"
            kind, xt, out = items2[k]
            assert oracle.rel_l2(out.cpu().numpy(), _ref(oracle, kind, xs2[k])) <= TOL
    finally:
        srv.close()


@pytest.mark.parametrize("max_wait_us", [50, -1])
def test_server_max_wait_bounds_a_lone_request(env, max_wait_us):
    """A lone request arriving while a long batch runs: with max_wait_us = 50
    it is launched (on another stream) before that batch completes, instead
    of waiting for min_batch requests; with no bound (-1) it waits for the GPU
    to go idle.  Both results match the oracle."""
    torch, dx, inputs, oracle = env
    head, _ = _make(env, 6700, reps=8, specs=[("dct2d", (4096, 4096))])
    lone, xl = _make(env, 6800, specs=[("dct2d", (64, 64))])
    print(f"[gpu] server max_wait_us={max_wait_us}", flush=True)
    srv = dx.Server(hbm_budget=2 << 30, max_inflight=64, nstreams=4, max_batch=16, min_batch=4,
                    max_wait_us=max_wait_us)
    try:
        for it in head + lone:   # warm-up: plans and workspace
            srv.submit((it[0], it[1], torch.empty_like(it[1])))
        srv.drain()
        t0 = srv.now() + 0.01
        th = [srv.submit(it, t0) for it in head]
        tl = srv.submit(lone[0], t0 + 3e-4)   # after the head batch has been launched
        srv.drain()
        sh = [srv.poll(t) for t in th]
        sl = srv.poll(tl)
        assert all(s["status"] == "OK" for s in sh) and sl["status"] == "OK"
        assert sl["batch_size"] == 1 and max(s["launch_s"] for s in sh) < sl["arrival_s"]
        head_done = min(s["done_s"] for s in sh)
        print(f"[gpu] lone request: arrival {sl['arrival_s'] - t0:.6f} s, launch {sl['launch_s'] - t0:.6f} s, "
              f"head batch done {head_done - t0:.6f} s", flush=True)
        if max_wait_us > 0:
            assert sl["launch_s"] < head_done, "the lone request waited for the running batch"
        else:
            assert sl["launch_s"] >= head_done, "the lone request was launched before the GPU went idle"
        assert oracle.rel_l2(lone[0][2].cpu().numpy(), oracle.dctn(xl[0])) <= TOL
    finally:
        srv.close()
