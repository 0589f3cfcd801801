"""GPU parity of the small-N matrix-core path (Y = C X C^T, batched) against
the FP64 oracle, through the C ABI.

Inputs: s * 10^u with u ~ U[-3, 3] and random signs (log-uniform magnitudes).
Tolerances (relative L2 per matrix, maximum over the batch): bf16x3 <= 2e-5,
scaled FP16 <= 1e-3 (the precision is the caller's explicit choice).  The FP32
FFT path is compared too, to the same tolerance."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL = {"bf16x3": 2e-5, "fp16": 1e-3}


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


def _per_matrix_err(y, ref):
    d = np.linalg.norm((y.astype(np.float64) - ref).reshape(len(ref), -1), axis=1)
    r = np.linalg.norm(ref.reshape(len(ref), -1), axis=1)
    return d / r


@pytest.mark.parametrize("prec", ["bf16x3", "fp16"])
@pytest.mark.parametrize("n", [16, 32, 64, 128])
@pytest.mark.parametrize("inverse,norm", [(False, "backward"), (False, "ortho"), (True, "backward"),
                                          (True, "ortho")])
def test_small_vs_oracle(env, n, prec, inverse, norm):
    torch, dx, inputs, oracle = env
    b = 37   # not a multiple of the 4 matrices per workgroup of n <= 32
    x = inputs.log_uniform_signed((b, n, n), 4000 + n)
    print(f"[gpu] dct2d_small n={n} prec={prec} inverse={inverse} norm={norm}", flush=True)
    y = dx.dct2d_small(torch.from_numpy(x).cuda(), prec, inverse, norm)
    torch.cuda.synchronize()
    f = oracle.idctn if inverse else oracle.dctn
    ref = f(x, norm, axes=(1, 2))
    err = _per_matrix_err(y.cpu().numpy(), ref)
    assert err.max() <= TOL[prec], f"n={n} {prec}: max rel L2 {err.max():.3e}"


@pytest.mark.parametrize("n", [16, 32, 64, 128])
def test_config4_batch_8192(env, n):
    """8192 matrices per launch: the whole batch against the oracle for n <= 64,
    512 random matrices at 128; both precisions; also against the FP32 FFT path
    (the batched three-stage kernels)."""
    torch, dx, inputs, oracle = env
    b = 8192
    x = inputs.log_uniform_signed((b, n, n), 4100 + n)
    xt = torch.from_numpy(x).cuda()
    idx = np.arange(b) if n <= 64 else np.sort(np.random.default_rng(n).choice(b, 512, replace=False))
    ref = oracle.dctn(x[idx], axes=(1, 2))
    fp32 = torch.empty_like(xt)
    dx.submit_batch([("dct2d", xt[i], fp32[i]) for i in idx.tolist()])
    for prec in ("bf16x3", "fp16"):
        print(f"[gpu] dct2d_small batch {b} n={n} prec={prec}", flush=True)
        y = dx.dct2d_small(xt, prec)
        torch.cuda.synchronize()
        err = _per_matrix_err(y.cpu().numpy()[idx], ref)
        assert err.max() <= TOL[prec], f"n={n} {prec}: max rel L2 {err.max():.3e}"
    e32 = _per_matrix_err(fp32.cpu().numpy()[idx], ref)
    assert e32.max() <= 1e-6


def test_small_deterministic_and_errors(env):
    torch, dx, inputs, _ = env
    x = torch.from_numpy(inputs.log_uniform_signed((9, 32, 32), 4200)).cuda()
    a = dx.dct2d_small(x, "bf16x3")
    b = dx.dct2d_small(x, "bf16x3")
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    bad = torch.zeros((4, 24, 24), device="cuda")
    out = torch.full_like(bad, 2.0)
    with pytest.raises(dx.DctxError):
        dx.dct2d_small(bad, out=out)
    torch.cuda.synchronize()
    assert bool((out == 2.0).all())
