"""fib_mlp_gradient_noalloc (the gradient for callers that cannot allocate)
against fib_mlp_gradient, through the C ABI.

Both run the same kernels with the same fixed-order reduction, so the
gradients and losses must agree bit for bit; the no-allocation entry point
keeps its per-chunk partials in the library's fixed per-device array, which
two calls in a row share (the second with a smaller batch reads only what it
wrote itself).  A batch beyond the array's capacity is refused before any
launch.
"""
import numpy as np
import pytest

from oracle import mlp as M
from paper_2107_07104_amd import fib as F

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    F.lib()


@pytest.mark.parametrize("sizes,act,batches", [([57, 128, 128, 57], "relu", (4000, 777)),
                                               ([5, 64, 64, 64, 4], "silu", (9000, 130))])
def test_noalloc_gradient_equals_the_allocating_entry_point(sizes, act, batches):
    print(f"[noalloc gradient] {sizes} {act} batches {batches}", flush=True)
    net = F.Mlp(sizes, act=act)
    rng = np.random.default_rng(21)
    params = [(W, 0.1 * rng.standard_normal(b.shape)) for W, b in M.init_params(sizes, seed=22)]
    net.set_params(M.flatten(params).astype(np.float32))
    n = net.n_params
    for B in batches:
        X = torch.as_tensor(rng.standard_normal((B, sizes[0])), dtype=torch.float32, device="cuda")
        T = torch.as_tensor(rng.standard_normal((B, sizes[-1])), dtype=torch.float32, device="cuda")
        g_ref, l_ref = net.gradient(X, T)
        g = torch.full((n,), float("nan"), device="cuda")
        loss = torch.full((1,), float("nan"), device="cuda")
        F.fib_mlp_gradient_noalloc(net.net, X.data_ptr(), T.data_ptr(), B, g.data_ptr(),
                                   loss.data_ptr())
        torch.cuda.synchronize()
        gr, ga = g_ref.cpu().numpy(), g.cpu().numpy()
        print(f"   B={B}: max |g - g_ref| {np.max(np.abs(ga - gr)):.1e}, loss {loss.item():.6e} "
              f"vs {l_ref.item():.6e}", flush=True)
        np.testing.assert_array_equal(ga, gr)
        np.testing.assert_array_equal(loss.cpu().numpy(), l_ref.cpu().numpy())
    # beyond the array's capacity: refused, nothing launched
    big = 5000 if sizes[0] == 57 else 20000
    Xb = torch.zeros((big, sizes[0]), device="cuda")
    Tb = torch.zeros((big, sizes[-1]), device="cuda")
    with pytest.raises(F.FibError) as err:
        F.fib_mlp_gradient_noalloc(net.net, Xb.data_ptr(), Tb.data_ptr(), big, 0, 0)
    assert err.value.code == F.FIB_EINVAL
    torch.cuda.synchronize()
    net.close()
