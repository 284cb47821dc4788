"""The recomputation checkpoint of the differentiable network contraction,
checked on the host: a segment whose replay is a plain torch CPU function must
give the gradients of running that function directly (no GPU, no library)."""

import torch

from paper_2410_02215_amd.autograd import _Segment


def _seg(x, y):
    # two outputs from two inputs, with a shared intermediate
    t = x * y.sum()
    return [t.exp() * 0.5, (t * y[:1]).sin()]


def test_segment_gradients_equal_the_direct_ones():
    g = torch.Generator().manual_seed(5)
    x0 = torch.randn(6, dtype=torch.float64, generator=g)
    y0 = torch.randn(6, dtype=torch.float64, generator=g)
    w0, w1 = torch.randn(6, dtype=torch.float64, generator=g), torch.randn(6, dtype=torch.float64, generator=g)
    # direct
    x, y = x0.clone().requires_grad_(True), y0.clone().requires_grad_(True)
    a, b = _seg(x, y)
    L = (a * w0).sum() + (b * w1).sum()
    gx, gy = torch.autograd.grad(L, [x, y])
    # through the checkpoint: outputs computed without a graph, replayed in backward
    x2, y2 = x0.clone().requires_grad_(True), y0.clone().requires_grad_(True)
    with torch.no_grad():
        outs = _seg(x2, y2)
    calls = []

    def replay(ins):
        calls.append(1)
        return _seg(*ins)

    a2, b2 = _Segment.apply(replay, outs, x2, y2)
    assert not calls  # the forward pass does not run the segment again
    assert torch.equal(a2, a.detach()) and torch.equal(b2, b.detach())
    L2 = (a2 * w0).sum() + (b2 * w1).sum()
    hx, hy = torch.autograd.grad(L2, [x2, y2])
    assert len(calls) == 1
    assert torch.allclose(hx, gx, rtol=1e-14, atol=0) and torch.allclose(hy, gy, rtol=1e-14, atol=0)


def test_segment_with_an_unused_output_and_a_constant_input():
    g = torch.Generator().manual_seed(6)
    x0 = torch.randn(4, dtype=torch.float64, generator=g)
    c = torch.randn(4, dtype=torch.float64, generator=g)  # does not require grad
    x = x0.clone().requires_grad_(True)
    with torch.no_grad():
        outs = _seg(x, c)
    a, b = _Segment.apply(lambda ins: _seg(*ins), outs, x, c)
    (gx,) = torch.autograd.grad(a.sum(), [x])  # b takes no part in the loss
    x3 = x0.clone().requires_grad_(True)
    (rx,) = torch.autograd.grad(_seg(x3, c)[0].sum(), [x3])
    assert torch.allclose(gx, rx, rtol=1e-14, atol=0)
