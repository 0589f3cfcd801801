"""GPU parity of the 3-D three-stage DCT-II / DCT-III against the FP64 oracle,
through the C ABI (via the thin Python binding).

Tolerance: relative L2 error <= 1e-6 over the compared outputs.  Every array
is compared whole against the oracle, 128^3 and 256^3 included (in the launch
configuration the benchmark uses)."""
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


def _run(env, fn, x_np, norm="backward"):
    torch, dx, _, _ = env
    print(f"[gpu] {fn} shape={x_np.shape} norm={norm}", flush=True)
    x = torch.from_numpy(x_np).cuda()
    y = getattr(dx, fn)(x, norm)
    torch.cuda.synchronize()
    return y.cpu().numpy()


REF = {"dct3d": "dctn", "idct3d": "idctn"}

SMALL = [(2, 2, 4), (3, 5, 6), (4, 6, 8), (8, 8, 8), (5, 9, 10), (2, 3, 4), (16, 12, 20),
         (15, 25, 12), (30, 18, 40), (64, 48, 36), (6, 4, 100), (40, 3, 64), (9, 50, 16), (32, 32, 32)]


@pytest.mark.parametrize("norm", ["backward", "ortho"])
@pytest.mark.parametrize("shape", SMALL)
@pytest.mark.parametrize("fn", ["dct3d", "idct3d"])
def test_small_full(env, fn, shape, norm):
    _, _, inputs, oracle = env
    x = inputs.uniform(shape, 3000 + sum(shape))
    y = _run(env, fn, x, norm)
    ref = getattr(oracle, REF[fn])(x, norm)
    err = oracle.rel_l2(y, ref)
    assert err <= TOL, f"{fn} {shape} {norm}: rel L2 {err:.3e}"


@pytest.mark.parametrize("fn", ["dct3d", "idct3d"])
def test_128_cubed_full(env, fn):
    """128^3, N(0,1), seed 2100: the whole output against the oracle."""
    _, _, inputs, oracle = env
    x = inputs.normal((128, 128, 128), 2100)
    y = _run(env, fn, x)
    ref = getattr(oracle, REF[fn])(x)
    err = oracle.rel_l2(y, ref)
    assert err <= TOL, f"{fn} 128^3: rel L2 {err:.3e}"


@pytest.mark.parametrize("fn", ["dct3d", "idct3d"])
def test_256_cubed_full(env, fn):
    """256^3, N(0,1), seed 2101: the whole output against the oracle, with the
    output NaN-poisoned first so every element must be written."""
    torch, dx, inputs, oracle = env
    n = 256
    x_np = inputs.normal((n, n, n), 2101)
    x = torch.from_numpy(x_np).cuda()
    y = torch.full_like(x, float("nan"))
    print(f"[gpu] {fn} 256^3 whole array", flush=True)
    getattr(dx, fn)(x, out=y)
    torch.cuda.synchronize()
    yn = y.cpu().numpy()
    assert np.isfinite(yn).all()
    err = oracle.rel_l2(yn, getattr(oracle, REF[fn])(x_np))
    assert err <= TOL, f"{fn} 256^3: whole-array rel L2 {err:.3e}"


@pytest.mark.parametrize("shape,norm", [((128, 128, 128), "backward"), ((48, 80, 96), "ortho"),
                                        ((25, 12, 30), "backward")])
def test_roundtrip(env, shape, norm):
    torch, dx, inputs, oracle = env
    x = inputs.uniform(shape, 3100 + sum(shape))
    xt = torch.from_numpy(x).cuda()
    back = dx.idct3d(dx.dct3d(xt, norm), norm).cpu().numpy()
    err = oracle.rel_l2(back, x)
    assert err <= TOL, f"roundtrip {shape} {norm}: rel L2 {err:.3e}"


@pytest.mark.parametrize("fn", ["dct3d", "idct3d"])
@pytest.mark.parametrize("shape", [(6, 10, 12), (64, 64, 64), (5, 9, 10)])
def test_every_output_written(env, fn, shape):
    """Outputs pre-filled with NaN: every element is written (write-once post)."""
    torch, dx, inputs, _ = env
    x = torch.from_numpy(inputs.normal(shape, 3200)).cuda()
    out = torch.full(shape, float("nan"), device="cuda")
    getattr(dx, fn)(x, out=out)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(out).all())


def test_deterministic(env):
    torch, dx, inputs, _ = env
    x = torch.from_numpy(inputs.normal((64, 96, 80), 3300)).cuda()
    a = dx.dct3d(x)
    b = dx.dct3d(x)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_unaligned_16B(env):
    """8-byte but not 16-byte aligned buffers take the generic row kernels."""
    torch, dx, inputs, oracle = env
    shape = (16, 24, 64)
    x_np = inputs.normal(shape, 3400)
    n = x_np.size
    xb = torch.zeros(n + 2, device="cuda")
    yb = torch.zeros(n + 2, device="cuda")
    x = xb[2:].view(shape)
    x.copy_(torch.from_numpy(x_np).cuda())
    y = yb[2:].view(shape)
    assert x.data_ptr() % 16 == 8
    dx.dct3d(x, out=y)
    torch.cuda.synchronize()
    assert oracle.rel_l2(y.cpu().numpy(), oracle.dctn(x_np)) <= TOL


ODD3 = [(4, 4, 5), (6, 10, 15), (8, 9, 25), (16, 12, 45), (3, 5, 3), (32, 24, 81), (5, 6, 2), (64, 64, 2),
        (64, 64, 75), (128, 128, 135)]


@pytest.mark.parametrize("norm", ["backward", "ortho"])
@pytest.mark.parametrize("shape", ODD3)
@pytest.mark.parametrize("fn", ["dct3d", "idct3d"])
def test_odd_and_two_last_dimension(env, fn, shape, norm):
    """Odd n3 (full-length row FFTs; the k3 = 0 column alone, with four
    outputs and no n3 - k3 partner) and n3 = 2 (a length-1 row FFT): whole
    arrays against the oracle, outputs NaN-poisoned."""
    torch, dx, inputs, oracle = env
    x_np = inputs.uniform(shape, 3600 + sum(shape))
    x = torch.from_numpy(x_np).cuda()
    y = torch.full_like(x, float("nan"))
    print(f"[gpu] {fn} odd {shape} {norm}", flush=True)
    getattr(dx, fn)(x, norm, out=y)
    torch.cuda.synchronize()
    yn = y.cpu().numpy()
    assert np.isfinite(yn).all()
    err = oracle.rel_l2(yn, getattr(oracle, REF[fn])(x_np, norm))
    assert err <= TOL, f"{fn} {shape} {norm}: rel L2 {err:.3e}"


@pytest.mark.parametrize("shape", [(4, 4, 7), (1, 4, 8), (4, 7, 8), (8192, 2, 4), (2, 16384, 4), (4, 4, 9375)])
def test_unsupported_shapes_enqueue_nothing(env, shape):
    torch, dx, _, _ = env
    x = torch.zeros(shape, device="cuda")
    y = torch.full(shape, 5.0, device="cuda")
    with pytest.raises(dx.DctxError):
        dx.dct3d(x, out=y)
    torch.cuda.synchronize()
    assert bool((y == 5.0).all())


@pytest.mark.parametrize("shape", [(64, 128, 40), (256, 64, 16), (128, 256, 100), (64, 64, 6), (256, 256, 36),
                                   (128, 64, 256)])
def test_fast_kernels_vs_oracle_and_general(env, shape):
    """Power-of-two n1, n2 in [64, 256] take the compile-time n2 / n1 kernels:
    the whole array against the oracle and against the run-time-schedule
    kernels (a handle created with DCTX_FAST=0)."""
    import os
    torch, dx, inputs, oracle = env
    x_np = inputs.normal(shape, 3500 + sum(shape))
    x = torch.from_numpy(x_np).cuda()
    fast = dx.Handle(0)
    os.environ["DCTX_FAST"] = "0"
    try:
        gen = dx.Handle(0)
        a = dx.dct3d(x, handle=gen)
        b = dx.idct3d(x, handle=gen)
    finally:
        del os.environ["DCTX_FAST"]
    print(f"[gpu] fast 3d {shape}", flush=True)
    c = dx.dct3d(x, handle=fast)
    d = dx.idct3d(x, handle=fast)
    torch.cuda.synchronize()
    assert oracle.rel_l2(c.cpu().numpy(), a.cpu().numpy()) <= TOL
    assert oracle.rel_l2(d.cpu().numpy(), b.cpu().numpy()) <= TOL
    assert oracle.rel_l2(c.cpu().numpy(), oracle.dctn(x_np)) <= TOL
    assert oracle.rel_l2(d.cpu().numpy(), oracle.idctn(x_np)) <= TOL


PLANE = [((128, 128, 128), None), ((64, 64, 64), None), ((64, 128, 100), None), ((256, 64, 40), None),
         ((128, 64, 256), None), ((64, 64, 6), None), ((64, 128, 2), None), ((256, 128, 10), None),
         ((128, 128, 128), {"DCTX_PLANE_CW": "64", "DCTX_PLANE_RW": "128", "DCTX_PLANE_BLOCK": "512"}),
         ((64, 64, 64), {"DCTX_PLANE_CW": "8", "DCTX_PLANE_RW": "16", "DCTX_PLANE_BLOCK": "512"})]


@pytest.mark.parametrize("shape,geo", PLANE)
def test_plane_route_vs_three_pass_and_oracle(env, shape, geo):
    """Two-pass route (DCTX_PLANE=1; even n3, power-of-two n1, n2 in [64, 256],
    n2 n3 <= 128^2): the plane pass (n3 and n2 FFTs of a plane in one
    workgroup) and the n1 pass.  Whole arrays, NaN-poisoned outputs, against
    the oracle and against the three-pass route (DCTX_PLANE=0 DCTX_FPLANE=0), in the default
    tile geometry and in others (one workgroup per plane; smaller tiles, 512
    threads)."""
    import os
    torch, dx, inputs, oracle = env
    x_np = inputs.normal(shape, 3700 + sum(shape))
    x = torch.from_numpy(x_np).cuda()
    os.environ["DCTX_PLANE"] = "0"
    os.environ["DCTX_FPLANE"] = "0"
    try:
        three = dx.Handle(0)
        a = dx.dct3d(x, handle=three)
        b = dx.idct3d(x, handle=three)
    finally:
        del os.environ["DCTX_PLANE"]
        del os.environ["DCTX_FPLANE"]
    geo = dict(geo or {}, DCTX_PLANE="1")
    for k, v in geo.items():
        os.environ[k] = v
    try:
        two = dx.Handle(0)
        print(f"[gpu] plane route {shape} {geo}", flush=True)
        c = torch.full_like(x, float("nan"))
        d = torch.full_like(x, float("nan"))
        dx.dct3d(x, out=c, handle=two)
        dx.idct3d(x, out=d, handle=two)
        two.profile(True)
        two.profile_read()
        dx.dct3d(x, out=c, handle=two)
        prof = two.profile_read()
        two.profile(False)
    finally:
        for k in geo:
            del os.environ[k]
    torch.cuda.synchronize()
    assert "dct3_plane" in prof and "dct3_rows" not in prof, f"{shape}: not on the plane route ({sorted(prof)})"
    cn, dn = c.cpu().numpy(), d.cpu().numpy()
    assert np.isfinite(cn).all() and np.isfinite(dn).all()
    assert oracle.rel_l2(cn, a.cpu().numpy()) <= TOL
    assert oracle.rel_l2(dn, b.cpu().numpy()) <= TOL
    assert oracle.rel_l2(cn, oracle.dctn(x_np)) <= TOL
    assert oracle.rel_l2(dn, oracle.idctn(x_np)) <= TOL


FPLANE = [(128, 128, 128), (64, 64, 64), (256, 128, 128), (64, 128, 64), (128, 64, 128), (256, 64, 64),
          (128, 128, 64)]


@pytest.mark.parametrize("shape", FPLANE)
def test_compile_time_plane_route(env, shape):
    """Compile-time two-pass route (the default for n2 in {64, 128}, n3 in
    {64, 128}, power-of-two n1 in [64, 256]): one workgroup per n1-plane runs
    the n3 row FFTs and the n2 FFTs with the packed half-spectrum plane in LDS,
    then the n1 pass.  Both directions on the route (per-kernel profile), whole
    NaN-poisoned outputs against the oracle and against the three-pass route
    (DCTX_FPLANE=0)."""
    import os
    torch, dx, inputs, oracle = env
    x_np = inputs.normal(shape, 3900 + sum(shape))
    x = torch.from_numpy(x_np).cuda()
    os.environ["DCTX_FPLANE"] = "0"
    try:
        three = dx.Handle(0)
        a = dx.dct3d(x, handle=three)
        b = dx.idct3d(x, handle=three)
    finally:
        del os.environ["DCTX_FPLANE"]
    two = dx.Handle(0)
    print(f"[gpu] compile-time plane route {shape}", flush=True)
    c = torch.full_like(x, float("nan"))
    d = torch.full_like(x, float("nan"))
    two.profile(True)
    two.profile_read()
    dx.dct3d(x, out=c, handle=two)
    dx.idct3d(x, out=d, handle=two)
    prof = two.profile_read()
    two.profile(False)
    torch.cuda.synchronize()
    assert {"dct3_plane", "idct3_plane"} <= set(prof), f"{shape}: not on the plane route ({sorted(prof)})"
    assert "dct3_rows" not in prof and "idct3_rows" not in prof and "dct3_mid" not in prof
    cn, dn = c.cpu().numpy(), d.cpu().numpy()
    assert np.isfinite(cn).all() and np.isfinite(dn).all()
    assert oracle.rel_l2(cn, a.cpu().numpy()) <= TOL
    assert oracle.rel_l2(dn, b.cpu().numpy()) <= TOL
    assert oracle.rel_l2(cn, oracle.dctn(x_np)) <= TOL
    assert oracle.rel_l2(dn, oracle.idctn(x_np)) <= TOL
    back = dx.idct3d(c, handle=two)
    torch.cuda.synchronize()
    assert oracle.rel_l2(back.cpu().numpy(), x_np) <= TOL
