"""GPU parity of the warm-start network kernels (BF16 MFMA) against the FP64 oracle.

Both sides see the same bf16-rounded operands, so only accumulation order and
the final rounding differ: bf16 outputs must agree within one bf16 ulp of the
oracle value, FP32 outputs within 1e-4 relative.
"""

import numpy as np
import pytest

import oracle as O
from paper_1210_2687_amd import admm as A
from gpu_util import announce

pytestmark = pytest.mark.gpu

BF16_ULP = 2.0 ** -8


def bf16(a):
    import torch
    return torch.tensor(np.asarray(a), dtype=torch.float32).to(torch.bfloat16).to(torch.float32).double().numpy()


def to_bf16_dev(a):
    import torch
    return torch.tensor(np.asarray(a), dtype=torch.float32).to(torch.bfloat16).cuda().contiguous()


def to_f32_dev(a):
    import torch
    return torch.tensor(np.asarray(a), dtype=torch.float32).cuda().contiguous()


def host(t):
    return t.detach().float().cpu().double().numpy()


def oracle_w(w):
    """[tap][co][ci] -> oracle layout [ky][kx][ci][co]."""
    cout, cin = w.shape[1], w.shape[2]
    return w.reshape(3, 3, cout, cin).transpose(0, 1, 3, 2)


def close_bf16(got, ref):
    refb = bf16(ref)
    err = np.abs(got - refb)
    tol = 2 * BF16_ULP * np.abs(refb) + 1e-6 * max(1.0, np.abs(refb).max())
    return np.all(err <= tol), float((err / np.maximum(np.abs(refb), 1e-3)).max())


def packed(w, cin_p, cout_p):
    import torch
    wf = torch.zeros(9 * 32 * 32, dtype=torch.bfloat16, device="cuda")
    wb = torch.zeros(9 * 32 * 32, dtype=torch.bfloat16, device="cuda")
    A.admm_conv3x3_pack_weights(to_f32_dev(w), cin_p, cout_p, wf, wb)
    return wf, wb


@pytest.mark.parametrize("cin,cout,N,H,W,relu,dil", [(8, 32, 2, 20, 37, 1, 1), (32, 32, 1, 33, 70, 1, 1),
                                                      (32, 16, 2, 17, 16, 0, 1), (16, 32, 1, 9, 130, 1, 1),
                                                      (8, 32, 2, 20, 37, 1, 2), (32, 32, 1, 33, 70, 1, 4),
                                                      (32, 16, 2, 17, 16, 0, 8)])
def test_conv_forward(cin, cout, N, H, W, relu, dil):
    import torch
    announce(f"conv fwd cin={cin} cout={cout} {N}x{H}x{W} dilation {dil}")
    g = np.random.default_rng(cin * 100 + cout)
    x = bf16(g.standard_normal((N, H, W, cin)))
    w = bf16(0.2 * g.standard_normal((9, cout, cin)))
    b = g.standard_normal(cout).astype(np.float32)
    wf, _ = packed(w, cin, cout)
    y = torch.zeros(N, H, W, cout, dtype=torch.bfloat16, device="cuda")
    A.admm_conv3x3_bf16_fwd(to_bf16_dev(x), N, H, W, cin, wf, to_f32_dev(b), cout, relu, None, y, dil=dil)
    torch.cuda.synchronize()
    ref = O.conv3x3_fwd(x, oracle_w(w), b, dil=dil)
    if relu:
        ref = O.relu(ref)
    ok, worst = close_bf16(host(y), ref)
    announce(f"  worst rel {worst:.2e}")
    assert ok


@pytest.mark.parametrize("cin,cout,N,H,W,dil", [(32, 32, 2, 19, 45, 1), (32, 16, 1, 24, 33, 1),
                                                 (32, 32, 2, 19, 45, 4), (32, 16, 1, 24, 33, 8)])
def test_conv_input_gradient_with_relu_gate(cin, cout, N, H, W, dil):
    import torch
    announce(f"conv dgrad cin={cin} cout={cout} dilation {dil}")
    g = np.random.default_rng(7 + cin + cout)
    w = bf16(0.2 * g.standard_normal((9, cout, cin)))
    dy = bf16(g.standard_normal((N, H, W, cout)))
    gate = bf16(g.standard_normal((N, H, W, cin)))
    _, wb = packed(w, cin, cout)
    dx = torch.zeros(N, H, W, cin, dtype=torch.bfloat16, device="cuda")
    A.admm_conv3x3_bf16_fwd(to_bf16_dev(dy), N, H, W, cout, wb, None, cin, 0, to_bf16_dev(gate), dx, dil=dil)
    torch.cuda.synchronize()
    ref = O.conv3x3_dgrad(dy, oracle_w(w), dil=dil) * (gate > 0)
    ok, worst = close_bf16(host(dx), ref)
    announce(f"  worst rel {worst:.2e}")
    assert ok


@pytest.mark.parametrize("cin,cout,N,H,W,chunk,dil", [(8, 32, 2, 21, 37, 256, 1), (32, 32, 1, 30, 70, 1024, 1),
                                                      (32, 16, 3, 16, 16, 96, 1), (8, 32, 2, 21, 37, 256, 2),
                                                      (32, 32, 1, 30, 70, 1024, 8), (32, 16, 3, 16, 16, 96, 4)])
def test_conv_weight_gradient(cin, cout, N, H, W, chunk, dil):
    import torch
    announce(f"conv wgrad cin={cin} cout={cout} chunk={chunk} dilation {dil}")
    g = np.random.default_rng(11 + cin + cout)
    x = bf16(g.standard_normal((N, H, W, cin)))
    dy = bf16(g.standard_normal((N, H, W, cout)))
    ws = torch.zeros(A.admm_conv3x3_bf16_wgrad_workspace(N, H, W, cin, cout, chunk) // 4 + 1,
                     dtype=torch.float32, device="cuda")
    dw = torch.zeros(9, cout, cin, dtype=torch.float32, device="cuda")
    db = torch.zeros(cout, dtype=torch.float32, device="cuda")
    A.admm_conv3x3_bf16_wgrad(to_bf16_dev(x), to_bf16_dev(dy), N, H, W, cin, cout, chunk, ws, dw, db, dil=dil)
    torch.cuda.synchronize()
    dwo, dbo = O.conv3x3_wgrad(x, dy, dil=dil)
    ref = dwo.transpose(0, 1, 3, 2).reshape(9, cout, cin)
    e = np.abs(host(dw) - ref).max() / np.abs(ref).max()
    eb = np.abs(host(db) - dbo).max() / np.abs(dbo).max()
    announce(f"  dw rel {e:.2e} db rel {eb:.2e}")
    assert e <= 1e-4 and eb <= 1e-4


def test_adam_matches_oracle():
    import torch
    g = np.random.default_rng(3)
    p = g.standard_normal(1000)
    m, v = np.zeros(1000), np.zeros(1000)
    pd, md, vd = to_f32_dev(p), to_f32_dev(m), to_f32_dev(v)
    for t in range(1, 6):
        grad = g.standard_normal(1000)
        A.admm_adam_step(pd, to_f32_dev(grad), md, vd, 1e-2, t)
        p, m, v = O.adam_step(p, grad, m, v, t, 1e-2)
    torch.cuda.synchronize()
    assert np.abs(host(pd) - p).max() <= 1e-5 * np.abs(p).max()


def test_warmstart_loss_input_output():
    import torch
    g = np.random.default_rng(5)
    N, H, W = 2, 13, 21
    y = g.standard_normal((N, H, W))
    m = (g.uniform(size=(N, H, W)) > 0.3).astype(np.uint8)
    emb = g.standard_normal((N, 4))
    x0 = torch.zeros(N, H, W, 8, dtype=torch.bfloat16, device="cuda")
    md = torch.tensor(m, device="cuda")
    A.admm_ws_input(to_f32_dev(y), md, to_f32_dev(emb), N, H, W, x0)
    xin = host(x0)
    assert np.allclose(xin[..., 0], bf16(m * y)) and np.array_equal(xin[..., 1], m.astype(float))
    assert np.allclose(xin[..., 2:6], bf16(np.broadcast_to(emb[:, None, None, :], (N, H, W, 4))))
    out = bf16(g.standard_normal((N, H, W, 16)))
    xt = g.standard_normal((N, H, W))
    pt = g.standard_normal((N, 2, H, W))
    dout = torch.zeros(N, H, W, 16, dtype=torch.bfloat16, device="cuda")
    lpart = torch.zeros((N * H * W + 255) // 256, dtype=torch.float32, device="cuda")
    A.admm_ws_loss(to_bf16_dev(out), to_f32_dev(y), md, to_f32_dev(xt), to_f32_dev(pt), N, H, W, 0.5, dout, lpart)
    e0 = m * y + out[..., 0] - xt
    e1, e2 = out[..., 1] - pt[:, 0], out[..., 2] - pt[:, 1]
    L = np.mean(e0 ** 2 + 0.5 * (e1 ** 2 + e2 ** 2))
    assert abs(host(lpart).sum() - L) <= 1e-4 * L
    gd = host(dout)
    npx = N * H * W
    assert np.allclose(gd[..., 0], bf16(2 * e0 / npx), rtol=2 * BF16_ULP, atol=1e-9)
    assert np.all(gd[..., 3:] == 0)
    xo = torch.zeros(N, H, W, dtype=torch.float32, device="cuda")
    po = torch.zeros(N, 2, H, W, dtype=torch.float32, device="cuda")
    A.admm_ws_output(to_bf16_dev(out), to_f32_dev(y), md, N, H, W, xo, po)
    assert np.allclose(host(xo), (m * y + out[..., 0]), atol=1e-5)
    assert np.allclose(host(po)[:, 1], out[..., 2], atol=1e-6)
