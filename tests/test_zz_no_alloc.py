"""cc_mlp_gradient_noalloc (the gradient whose per-wave partials live in the
library's static device array) against cc_mlp_gradient, through the C ABI:
two calls in a row, the second with fewer rows, each compared with the
allocating entry point on the same rows.  The same kernels and summation
order run in both, so the results agree to the last bit; the test allows
float32 rounding (1e-6 relative) all the same."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from ccscenes import mlp_init

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def cg():
    import paper_2510_12053_amd.ccgpu as cg
    cg.lib()
    return cg


def _case(rng, N, B):
    X = torch.tensor(rng.normal(size=(N, 16)).astype(np.float32), device=DEV)
    T = torch.tensor(rng.normal(scale=0.1, size=(N, 3)).astype(np.float32), device=DEV)
    idx = torch.tensor(rng.permutation(N)[:B].astype(np.int32), device=DEV)
    return X, T, idx


def test_noalloc_gradient_matches_allocating_entry_point(cg):
    stream = torch.cuda.Stream(device=DEV)
    ctx = cg.cc_create(0, stream)
    try:
        rng = np.random.default_rng(11)
        theta = (mlp_init(5) + 0.05 * rng.normal(size=cg.MLP_NPARAM)).astype(np.float32)
        cg.cc_mlp_set(ctx, theta, rng.normal(size=16).astype(np.float32),
                      rng.uniform(0.5, 2.0, size=16).astype(np.float32))
        # many rows (every wave of the grid writes partials), then few (the
        # second call must not see the first call's partials)
        for N, B in ((40000, 20000), (600, 37)):
            X, T, idx = _case(rng, N, B)
            with torch.cuda.stream(stream):
                g_ref, loss_ref = cg.cc_mlp_gradient(ctx, X, T, idx)
                g = torch.full((cg.MLP_NPARAM,), float("nan"), dtype=torch.float32, device=DEV)
                loss = torch.full((1,), float("nan"), dtype=torch.float32, device=DEV)
                cg.cc_mlp_gradient_noalloc(ctx, X, T, idx, g, loss)
            stream.synchronize()
            a, b = g.cpu().numpy(), g_ref.cpu().numpy()
            assert np.all(np.isfinite(a))
            np.testing.assert_allclose(a, b, rtol=1e-6, atol=1e-6 * np.abs(b).max())
            assert abs(float(loss.cpu()[0]) - loss_ref) <= 1e-6 * abs(loss_ref)
            print(f"rows {B}: max |dg| = {np.abs(a - b).max():.3e}, loss {loss_ref:.6e}", flush=True)
        # sizes beyond the stated limit are refused, nothing is launched
        X, T, idx = _case(rng, 64, 16)
        g = torch.zeros(cg.MLP_NPARAM, dtype=torch.float32, device=DEV)
        st = cg._ml().cc_mlp_gradient_noalloc(ctx.handle, cg._dptr(X, "float32"), cg._dptr(T, "float32"),
                                              cg._dptr(idx, "int32"), 0, cg._dptr(g, "float32"), None)
        assert st == -1                       # CC_E_INVALID_ARG
        assert b"B must be" in cg.lib().cc_last_error(ctx.handle)
    finally:
        cg.cc_destroy(ctx)
