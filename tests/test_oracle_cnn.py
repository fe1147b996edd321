"""Pins for oracle/cnn.py: torch CPU library routines and finite differences."""

import numpy as np
import pytest
import torch

import oracle as O


def _rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


def test_conv_fwd_matches_torch_conv2d():
    x = _rand((2, 6, 7, 3), 0)
    w = _rand((3, 3, 3, 5), 1)
    b = _rand((5,), 2)
    ref = torch.nn.functional.conv2d(
        torch.from_numpy(x).permute(0, 3, 1, 2), torch.from_numpy(w).permute(3, 2, 0, 1),
        torch.from_numpy(b), padding=1).permute(0, 2, 3, 1).numpy()
    np.testing.assert_allclose(O.conv3x3_fwd(x, w, b), ref, atol=1e-12)


def test_conv_grads_match_torch_autograd():
    x = torch.from_numpy(_rand((2, 5, 6, 4), 3)).requires_grad_()
    w = torch.from_numpy(_rand((3, 3, 4, 3), 4)).requires_grad_()
    b = torch.from_numpy(_rand((3,), 5)).requires_grad_()
    R = torch.from_numpy(_rand((2, 5, 6, 3), 6))
    y = torch.nn.functional.conv2d(x.permute(0, 3, 1, 2), w.permute(3, 2, 0, 1), b, padding=1)
    (y.permute(0, 2, 3, 1) * R).sum().backward()
    np.testing.assert_allclose(O.conv3x3_dgrad(R.numpy(), w.detach().numpy()), x.grad.numpy(), atol=1e-12)
    dw, db = O.conv3x3_wgrad(x.detach().numpy(), R.numpy())
    np.testing.assert_allclose(dw, w.grad.numpy(), atol=1e-12)
    np.testing.assert_allclose(db, b.grad.numpy(), atol=1e-12)


def test_conv_grads_central_differences():
    x = _rand((1, 4, 5, 2), 7)
    w = _rand((3, 3, 2, 3), 8)
    R = _rand((1, 4, 5, 3), 9)
    L = lambda xx, ww: np.sum(O.conv3x3_fwd(xx, ww) * R)
    dx = O.conv3x3_dgrad(R, w)
    dw, _ = O.conv3x3_wgrad(x, R)
    h = 1e-6
    g = np.random.default_rng(10)
    for _ in range(6):
        idx = tuple(int(g.integers(0, s)) for s in x.shape)
        e = np.zeros_like(x)
        e[idx] = h
        assert abs((L(x + e, w) - L(x - e, w)) / (2 * h) - dx[idx]) < 1e-7
        idw = tuple(int(g.integers(0, s)) for s in w.shape)
        e = np.zeros_like(w)
        e[idw] = h
        assert abs((L(x, w + e) - L(x, w - e)) / (2 * h) - dw[idw]) < 1e-7


@pytest.mark.parametrize("d", [2, 3])
def test_dilated_conv_and_grads_match_torch(d):
    x = torch.from_numpy(_rand((2, 9, 11, 3), 20 + d)).requires_grad_()
    w = torch.from_numpy(_rand((3, 3, 3, 4), 30 + d)).requires_grad_()
    b = torch.from_numpy(_rand((4,), 40 + d)).requires_grad_()
    R = torch.from_numpy(_rand((2, 9, 11, 4), 50 + d))
    y = torch.nn.functional.conv2d(x.permute(0, 3, 1, 2), w.permute(3, 2, 0, 1), b, padding=d, dilation=d)
    np.testing.assert_allclose(O.conv3x3_fwd(x.detach().numpy(), w.detach().numpy(), b.detach().numpy(), dil=d),
                               y.permute(0, 2, 3, 1).detach().numpy(), atol=1e-12)
    (y.permute(0, 2, 3, 1) * R).sum().backward()
    np.testing.assert_allclose(O.conv3x3_dgrad(R.numpy(), w.detach().numpy(), dil=d), x.grad.numpy(), atol=1e-12)
    dw, db = O.conv3x3_wgrad(x.detach().numpy(), R.numpy(), dil=d)
    np.testing.assert_allclose(dw, w.grad.numpy(), atol=1e-12)
    np.testing.assert_allclose(db, b.grad.numpy(), atol=1e-12)


def test_dilated_conv_is_plain_conv_with_zero_stuffed_kernel():
    # a 3x3 kernel at dilation 2 is the 5x5 kernel with the taps at even offsets,
    # written here as the sum of two dilation-1 convolutions of shifted inputs
    x = _rand((1, 8, 10, 2), 60)
    w = _rand((3, 3, 2, 3), 61)
    y2 = O.conv3x3_fwd(x, w, dil=2)
    xp = np.pad(x, ((0, 0), (2, 2), (2, 2), (0, 0)))
    ref = np.zeros_like(y2)
    for ky in range(3):
        for kx in range(3):
            ref += xp[:, 2 * ky:2 * ky + 8, 2 * kx:2 * kx + 10, :] @ w[ky, kx]
    np.testing.assert_allclose(y2, ref, atol=1e-12)
    # brute force at one output pixel
    r, c = 3, 4
    v = sum(x[0, r + 2 * (ky - 1), c + 2 * (kx - 1)] @ w[ky, kx] for ky in range(3) for kx in range(3)
            if 0 <= r + 2 * (ky - 1) < 8 and 0 <= c + 2 * (kx - 1) < 10)
    np.testing.assert_allclose(y2[0, r, c], v, atol=1e-12)


def test_adam_first_step_closed_form_and_torch():
    g = np.array([0.3, -2.0, 1e-3])
    p0 = np.array([1.0, 2.0, 3.0])
    p1, m1, v1 = O.adam_step(p0, g, np.zeros(3), np.zeros(3), 1, lr=0.1)
    # bias-corrected first step moves each weight by lr * g / (|g| + eps)
    np.testing.assert_allclose(p1, p0 - 0.1 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    # several steps against torch.optim.Adam
    pt = torch.nn.Parameter(torch.from_numpy(p0.copy()))
    opt = torch.optim.Adam([pt], lr=0.05)
    p, m, v = p0.copy(), np.zeros(3), np.zeros(3)
    for t in range(1, 6):
        grad = np.sin(p * t)
        pt.grad = torch.from_numpy(grad.copy())
        opt.step()
        p, m, v = O.adam_step(p, grad, m, v, t, lr=0.05)
    np.testing.assert_allclose(p, pt.detach().numpy(), rtol=1e-12)
