"""The allocation-free entry point qb_mlp_grad_noalloc against qb_mlp_grad
(same kernels, same fixed summation order: bit-identical gradient and loss)
on two calls in a row, the second with a smaller batch, so that the static
scratch array still holds the first call's rows; and the size limit."""
import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda"


def qb():
    from paper_2502_13947_amd import qb as m
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return m


def _case(B, seed):
    rng = np.random.default_rng(seed)
    feat = oracle.bf16(rng.normal(0, 1, size=(B, 8)).astype(np.float32)).reshape(B, 8)
    lab = (rng.random(B) < 0.3).astype(np.uint8)
    W = oracle.bf16(rng.normal(0, 0.3, size=oracle.NPARAM).astype(np.float32))
    return (torch.as_tensor(feat.view(np.int16), device=DEV), torch.as_tensor(lab, device=DEV),
            torch.as_tensor(W.view(np.int16), device=DEV))


def test_mlp_grad_noalloc_equals_workspace_version_on_two_calls():
    for B, seed in ((qb().MLP_GRAD_NOALLOC_MAX_B, 1), (1000, 2)):
        print("no-alloc grad", B, flush=True)
        feat, lab, W = _case(B, seed)
        g0 = torch.zeros(oracle.NPARAM, dtype=torch.float32, device=DEV)
        l0 = torch.zeros(1, dtype=torch.float32, device=DEV)
        work = torch.zeros(qb().mlp_train_workspace(B), dtype=torch.uint8, device=DEV)
        qb().mlp_grad(feat, lab, W, g0, l0, work)
        g1 = torch.full((oracle.NPARAM,), float("nan"), dtype=torch.float32, device=DEV)
        l1 = torch.full((1,), float("nan"), dtype=torch.float32, device=DEV)
        qb().mlp_grad_noalloc(feat, lab, W, g1, l1)
        torch.cuda.synchronize()
        assert (g0.cpu().numpy().view(np.uint32) == g1.cpu().numpy().view(np.uint32)).all(), B
        assert l0.item() == l1.item(), B
        # and within the oracle's FP64 gradient on the same FP32 forward pass
        go, lo = oracle.mlp_grad(W.cpu().numpy().view(np.uint16), feat.cpu().numpy().view(np.uint16),
                                 lab.cpu().numpy())
        assert np.abs(g1.cpu().numpy().astype(np.float64) - go).max() <= 1e-4 * np.abs(go).max() + 1e-8, B
        assert abs(l1.item() - lo) <= 1e-5 * max(1.0, abs(lo)), B


def test_mlp_grad_noalloc_rejects_batches_beyond_its_array():
    B = qb().MLP_GRAD_NOALLOC_MAX_B + 1
    feat, lab, W = _case(B, 3)
    g = torch.zeros(oracle.NPARAM, dtype=torch.float32, device=DEV)
    with pytest.raises(qb().QBError) as ei:
        qb().mlp_grad_noalloc(feat, lab, W, g, None)
    assert ei.value.status == -5
