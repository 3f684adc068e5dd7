"""The selector gradient through the entry point that allocates nothing
(nnc_mlp_grad_static, a fixed per-device workspace inside the library) against
the same gradient with a caller-given workspace (nnc_mlp_grad), bit for bit, on
two calls in a row, the second with a smaller batch; and the size limit."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nnc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_18314_amd import binding
    binding.load()
    return binding


def _batch(g, B):
    X = torch.from_numpy(g.standard_normal((B, 6)).astype(np.float32)).cuda()
    y = torch.from_numpy(g.integers(0, 2, B).astype(np.int32)).cuda()
    w = torch.from_numpy((g.random(B) + 0.1).astype(np.float32)).cuda()
    return X, y, w


def test_static_workspace_gradient_equals_the_workspace_call(nnc):
    g = np.random.default_rng(11)
    p = torch.from_numpy((0.1 * g.standard_normal(nnc.SELECTOR_PARAMS)).astype(np.float32)).cuda()
    for B in (nnc.MLP_STATIC_MAX_B, 3000, 700):
        X, y, w = _batch(g, B)
        l0, g0 = nnc.mlp_grad(p, X, y, w)
        l1, g1 = nnc.mlp_grad_static(p, X, y, w)
        torch.cuda.synchronize()
        assert torch.equal(l0, l1), B
        assert torch.equal(g0, g1), B
        assert torch.isfinite(g1).all()


def test_static_workspace_rejects_oversized_batches(nnc):
    g = np.random.default_rng(12)
    p = torch.zeros(nnc.SELECTOR_PARAMS, dtype=torch.float32, device="cuda")
    X, y, w = _batch(g, nnc.MLP_STATIC_MAX_B + 1)
    with pytest.raises(nnc.NNCError) as ei:
        nnc.mlp_grad_static(p, X, y, w)
    assert ei.value.code == nnc.NNC_E_INVAL
