"""Surrogate-network kernels (include/fdtd_nn.h) against torch CPU references.

Kernel tests feed BF16-representable inputs, so a kernel differs from the
FP64 reference only by its FP32 accumulation order (and by the final BF16
rounding where it writes BF16, which is checked bit-exactly against the
kernel's own FP32 value).  The U-Net test compares the assembled network with
a torch CPU autograd model of the same arithmetic: FP32 layers, activations
rounded to BF16 after each ReLU (straight-through in the backward).
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
import torch.nn.functional as Fn  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nn():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2203_01462_amd import nn as m
    return m


def bf16_round(t):
    return t.float().to(torch.bfloat16).to(torch.float32)


def bits(t):
    """FP32 CPU tensor (BF16-representable) -> int16 bit patterns on the GPU."""
    return t.float().to(torch.bfloat16).view(torch.int16).cuda()


def unbits(b):
    return b.cpu().view(torch.bfloat16).to(torch.float32)


def rel(a, b):
    a, b = np.asarray(a, np.float64).ravel(), np.asarray(b, np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def to_cn(x):  # [N][C][H][W] -> [C][N][H][W]
    return x.permute(1, 0, 2, 3).contiguous()


def to_krsc(wt):  # torch [cout][cin][3][3] -> the library's [cout][3][3][cin], flattened per cout
    return wt.permute(0, 2, 3, 1).reshape(wt.shape[0], -1).contiguous()


def from_krsc(flat, cout, cin):
    return flat.view(cout, 3, 3, cin).permute(0, 3, 1, 2)


CONV_CASES = [
    # generic kernel: ragged pixel tiles, cout across two 64-tiles, K not a multiple of 16
    (3, 5, 70, 13, 11),
    (2, 40, 33, 16, 16),
    (1, 1, 32, 8, 8),
    (4, 96, 32, 24, 24),
    # LDS-tiled matrix-core kernel (cin % 32 == 0, h and w multiples of 16):
    # 32- and 64-channel output tiles, ragged cout, several channel chunks,
    # non-square images, the U-Net's deepest shape
    (2, 32, 64, 16, 16),
    (3, 64, 70, 32, 16),
    (2, 96, 32, 16, 48),
    (1, 32, 20, 16, 16),
    (2, 256, 256, 16, 16),
    # one input channel (the network's first layer): the direct forward kernel;
    # the weight gradient's one-channel kernel (h % 8, w % 64, cout <= 32,
    # a ragged last group of eight channels) or the generic one
    (2, 1, 32, 16, 64),
    (3, 1, 20, 8, 128),
    (1, 1, 48, 9, 70),
]


@pytest.mark.parametrize("n,cin,cout,h,w", CONV_CASES)
def test_conv_forward(nn, n, cin, cout, h, w):
    g = torch.Generator().manual_seed(n * 1000 + cin)
    x = bf16_round(torch.randn(n, cin, h, w, generator=g))
    wt = bf16_round(torch.randn(cout, cin, 3, 3, generator=g) / math.sqrt(cin * 9))
    b = torch.randn(cout, generator=g)
    ref = Fn.conv2d(x.double(), wt.double(), b.double(), padding=1)
    z = torch.empty(cout * n * h * w, dtype=torch.float32, device="cuda")
    a = torch.empty(cout * n * h * w, dtype=torch.int16, device="cuda")
    nn.conv3x3(bits(to_cn(x)), bits(to_krsc(wt)), b.cuda(), n, cin, cout, h, w, z=z, a=a)
    torch.cuda.synchronize()
    zc = z.cpu().view(cout, n, h, w).permute(1, 0, 2, 3)
    err = (zc.double() - ref).abs().max().item()
    scale = Fn.conv2d(x.abs().double(), wt.abs().double(), padding=1).max().item()
    assert err <= 2e-6 * scale, (err, scale)
    # fused ReLU + BF16: bit-exact against rounding the kernel's own FP32 output
    assert torch.equal(a.cpu(), bits(torch.relu(z.cpu())).cpu())


def test_conv_only_activation_output(nn):
    n, cin, cout, h, w = 2, 8, 16, 9, 9
    g = torch.Generator().manual_seed(7)
    x = bf16_round(torch.randn(n, cin, h, w, generator=g))
    wt = bf16_round(torch.randn(cout, cin, 3, 3, generator=g))
    z = torch.empty(cout * n * h * w, device="cuda")
    a1 = torch.empty(cout * n * h * w, dtype=torch.int16, device="cuda")
    a2 = torch.empty_like(a1)
    xb, wb = bits(to_cn(x)), bits(to_krsc(wt))
    nn.conv3x3(xb, wb, None, n, cin, cout, h, w, z=z, a=a1)
    nn.conv3x3(xb, wb, None, n, cin, cout, h, w, a=a2)
    torch.cuda.synchronize()
    assert torch.equal(a1.cpu(), a2.cpu())


@pytest.mark.parametrize("n,cin,cout,h,w", CONV_CASES)
def test_conv_backward(nn, n, cin, cout, h, w):
    g = torch.Generator().manual_seed(n * 1000 + cout)
    x = bf16_round(torch.randn(n, cin, h, w, generator=g))
    wt = bf16_round(torch.randn(cout, cin, 3, 3, generator=g) / math.sqrt(cin * 9))
    dz = bf16_round(torch.randn(n, cout, h, w, generator=g))
    xd = x.double().requires_grad_()
    wd = wt.double().requires_grad_()
    bd = torch.zeros(cout, dtype=torch.float64, requires_grad=True)
    Fn.conv2d(xd, wd, bd, padding=1).backward(dz.double())
    dx = torch.empty(cin * n * h * w, device="cuda")
    dw = torch.empty(cout * cin * 9, device="cuda")
    db = torch.empty(cout, device="cuda")
    wrot = torch.empty(cout * cin * 9, dtype=torch.int16, device="cuda")
    work = torch.empty(nn.wgrad_work(n, cin, cout, h, w), device="cuda")
    xb, dzb, wb = bits(to_cn(x)), bits(to_cn(dz)), bits(to_krsc(wt))
    nn.conv3x3_dgrad(dzb, wb, wrot, dx, n, cin, cout, h, w)
    nn.conv3x3_wgrad(xb, dzb, dw, db, work, n, cin, cout, h, w)
    torch.cuda.synchronize()
    dxc = dx.cpu().view(cin, n, h, w).permute(1, 0, 2, 3).double()
    sx = Fn.conv_transpose2d(dz.abs().double(), wt.abs().double(), padding=1).max().item()
    assert (dxc - xd.grad).abs().max().item() <= 2e-6 * sx
    sw = (dz.abs().sum() * x.abs().max()).item()
    assert (from_krsc(dw.cpu(), cout, cin).double() - wd.grad).abs().max().item() <= 2e-6 * sw
    assert np.allclose(db.cpu().double().numpy(), bd.grad.numpy(), rtol=1e-6, atol=1e-5)


@pytest.mark.parametrize("n,cin,cout,h,w", [
    # (the data gradient is a convolution from cout to cin channels)
    (3, 5, 70, 13, 11),     # generic kernel
    (2, 32, 64, 64, 64),    # tiled, 32-channel output tile
    (2, 96, 64, 32, 64),    # tiled, 64-channel output tiles, a ragged one
    (2, 32, 128, 32, 32),   # pipelined deep-layer variant, 32-channel tile
    (2, 256, 256, 16, 16),  # pipelined deep-layer variant
])
def test_dgrad_relu_fused_bit_exact(nn, n, cin, cout, h, w):
    """The data gradient with the ReLU backward of the layer below fused in
    gives the BF16 values of the two separate calls, bit for bit."""
    g = torch.Generator().manual_seed(31 + cin)
    wt = bf16_round(torch.randn(cout, cin, 3, 3, generator=g) / math.sqrt(cin * 9))
    dz = bf16_round(torch.randn(n, cout, h, w, generator=g))
    act = torch.relu(torch.randn(n, cin, h, w, generator=g))
    ab, dzb, wb = bits(to_cn(act)), bits(to_cn(dz)), bits(to_krsc(wt))
    wrot = torch.empty(cout * cin * 9, dtype=torch.int16, device="cuda")
    dx = torch.empty(cin * n * h * w, device="cuda")
    sep = torch.empty(cin * n * h * w, dtype=torch.int16, device="cuda")
    fused = torch.full_like(sep, 0x7fff)
    nn.conv3x3_dgrad(dzb, wb, wrot, dx, n, cin, cout, h, w)
    nn.relu_bf16_backward(ab, dx, sep)
    nn.conv3x3_dgrad_relu(dzb, wb, wrot, ab, fused, n, cin, cout, h, w)
    torch.cuda.synchronize()
    assert torch.equal(fused.cpu(), sep.cpu())
    assert (sep.cpu() == 0).float().mean().item() > 0.3  # the mask did zero entries


def test_rot_weights_all_layers_match_per_call_turn(nn):
    """Several layers' weights turned in one launch (fdtd_nn_rot_weights)
    land where the per-call turn of each data gradient puts them, so a data
    gradient given the turned weights (wt = NULL) is the same, bit for bit;
    entries between the layers are left alone."""
    g = torch.Generator().manual_seed(53)
    layers, ws, o = [], [], 0
    for cin, cout in [(5, 70), (32, 64), (96, 64), (256, 256), (64, 1)]:
        o = (o + 7) // 8 * 8 + 3 * 8  # gaps between the layers
        layers.append((cin, cout, o))
        ws.append(bf16_round(torch.randn(cout, cin, 3, 3, generator=g) / math.sqrt(cin * 9)))
        o += cout * cin * 9
    flat = torch.zeros(o, dtype=torch.int16)
    for (cin, cout, off), wt in zip(layers, ws):
        flat[off:off + cout * cin * 9] = bits(to_krsc(wt)).reshape(-1).cpu()
    w = flat.cuda()
    wrot = torch.full((o,), 0x1234, dtype=torch.int16, device="cuda")
    nn.rot_weights(layers, w, wrot)
    used = torch.zeros(o, dtype=torch.bool)
    for (cin, cout, off), wt in zip(layers, ws):
        m = cout * cin * 9
        one = torch.empty(m, dtype=torch.int16, device="cuda")
        n, h, wd = 2, 16, 24
        dz = bits(to_cn(bf16_round(torch.randn(n, cout, h, wd, generator=g))))
        dx1 = torch.empty(cin * n * h * wd, device="cuda")
        dx2 = torch.empty_like(dx1)
        nn.conv3x3_dgrad(dz, w[off:off + m], one, dx1, n, cin, cout, h, wd)
        nn.conv3x3_dgrad(dz, None, wrot[off:off + m], dx2, n, cin, cout, h, wd)
        torch.cuda.synchronize()
        assert torch.equal(wrot[off:off + m].cpu(), one.cpu())
        assert torch.equal(dx1.cpu(), dx2.cpu())
        used[off:off + m] = True
    assert bool((wrot.cpu()[~used] == 0x1234).all())
    with pytest.raises(nn.FDTDError):
        nn.rot_weights([(0, 4, 0)], w, wrot)
    with pytest.raises(nn.FDTDError):
        nn.rot_weights([(1, 1, 0)] * 33, w, wrot)


@pytest.mark.parametrize("n,cin,cout,h,w", [(4, 32, 32, 32, 32), (2, 64, 96, 16, 32), (7, 32, 16, 8, 16),
                                             (4, 1, 32, 16, 128)])
def test_wgrad_contiguous_bias_single_reduction(nn, n, cin, cout, h, w):
    """Weight and bias gradients in one buffer ([dw | db], the network's
    parameter layout) take one reduction over both; the values equal those
    written to separate buffers, bit for bit."""
    g = torch.Generator().manual_seed(41 + cout)
    x = bits(to_cn(bf16_round(torch.randn(n, cin, h, w, generator=g))))
    dz = bits(to_cn(bf16_round(torch.randn(n, cout, h, w, generator=g))))
    m = cout * cin * 9
    work = torch.empty(nn.wgrad_work(n, cin, cout, h, w), device="cuda")
    both = torch.full((m + cout,), float("nan"), device="cuda")
    dw = torch.empty(m, device="cuda")
    db = torch.empty(cout, device="cuda")
    nn.conv3x3_wgrad(x, dz, both[:m], both[m:], work, n, cin, cout, h, w)
    nn.conv3x3_wgrad(x, dz, dw, db, work, n, cin, cout, h, w)
    torch.cuda.synchronize()
    assert torch.equal(both[:m].cpu(), dw.cpu()) and torch.equal(both[m:].cpu(), db.cpu())
    ref = dz.cpu().view(torch.bfloat16).double().view(cout, -1).sum(1)
    assert np.allclose(db.cpu().double().numpy(), ref.numpy(), rtol=1e-6, atol=1e-4)


@pytest.mark.parametrize("n,cin,cout,h,w,shift", [
    (9, 3, 5, 40, 40, 0),     # generic kernel, several pixel ranges, a ragged last one
    (5, 32, 16, 32, 32, 0),   # tiled kernel, one pixel tile per partial sum
    (7, 64, 96, 24, 48, 0),   # tiled, ragged output-channel tile, 24 = 3 x 8 rows
    (5, 32, 16, 32, 32, 1),   # dz not 16-byte aligned: the generic kernel with the tiled plan's split count
])
def test_wgrad_many_splits(nn, n, cin, cout, h, w, shift):
    g = torch.Generator().manual_seed(3 + cin)
    x = bf16_round(torch.randn(n, cin, h, w, generator=g))
    dz = bf16_round(torch.randn(n, cout, h, w, generator=g))
    wd = torch.zeros(cout, cin, 3, 3, dtype=torch.float64, requires_grad=True)
    bd = torch.zeros(cout, dtype=torch.float64, requires_grad=True)
    Fn.conv2d(x.double(), wd, bd, padding=1).backward(dz.double())
    assert nn.wgrad_work(n, cin, cout, h, w) >= 2 * cout * cin * 9
    dw = torch.empty(cout * cin * 9, device="cuda")
    db = torch.empty(cout, device="cuda")
    work = torch.empty(nn.wgrad_work(n, cin, cout, h, w), device="cuda")
    dzb = bits(to_cn(dz)).reshape(-1)
    if shift:
        buf = torch.zeros(dzb.numel() + shift, dtype=torch.int16, device="cuda")
        buf[shift:] = dzb
        dzb = buf[shift:]
    nn.conv3x3_wgrad(bits(to_cn(x)), dzb, dw, db, work, n, cin, cout, h, w)
    torch.cuda.synchronize()
    sw = (dz.abs().sum() * x.abs().max()).item()
    assert (from_krsc(dw.cpu(), cout, cin).double() - wd.grad).abs().max().item() <= 2e-6 * sw
    assert np.allclose(db.cpu().double().numpy(), bd.grad.numpy(), rtol=1e-6, atol=1e-4)


def test_misaligned_weights_take_the_generic_kernel(nn):
    """A weight pointer that is not 16-byte aligned must still give the same
    convolution (the tiled kernel needs aligned 16-byte weight rows)."""
    n, cin, cout, h, w = 2, 32, 48, 16, 16
    g = torch.Generator().manual_seed(21)
    x = bf16_round(torch.randn(n, cin, h, w, generator=g))
    wt = bf16_round(torch.randn(cout, cin, 3, 3, generator=g) / math.sqrt(cin * 9))
    flat = bits(to_krsc(wt)).reshape(-1)
    shifted = torch.zeros(flat.numel() + 1, dtype=torch.int16, device="cuda")
    shifted[1:] = flat
    za = torch.empty(cout * n * h * w, device="cuda")
    zb = torch.empty_like(za)
    xb = bits(to_cn(x))
    nn.conv3x3(xb, flat, None, n, cin, cout, h, w, z=za)
    nn.conv3x3(xb, shifted[1:], None, n, cin, cout, h, w, z=zb)
    torch.cuda.synchronize()
    ref = Fn.conv2d(x.double(), wt.double(), padding=1)
    scale = Fn.conv2d(x.abs().double(), wt.abs().double(), padding=1).max().item()
    for z in (za, zb):
        zc = z.cpu().view(cout, n, h, w).permute(1, 0, 2, 3).double()
        assert (zc - ref).abs().max().item() <= 2e-6 * scale


def test_bf16_conversions_bit_exact(nn):
    g = torch.Generator().manual_seed(11)
    x = torch.cat([torch.randn(10000, generator=g) * 10 ** torch.randint(-30, 30, (10000,), generator=g).float(),
                   torch.tensor([0.0, -0.0, 1.0, 1.00390625, 1.005859375, 1.0078125, -2.5, 3.4e38, -3.4e38,
                                 float("inf"), float("-inf"), 1e-40, -1e-42])])
    # ties: values exactly halfway between BF16 neighbours round to even
    k = torch.arange(1, 2001, dtype=torch.int32) << 16
    ties = torch.cat([(k | 0x8000), ((k + 0x3F000000) | 0x8000)]).view(torch.float32)
    x = torch.cat([x, ties, -ties]).contiguous()
    y = nn.to_bf16(x.cuda())
    torch.cuda.synchronize()
    assert torch.equal(y.cpu(), x.to(torch.bfloat16).view(torch.int16))
    back = nn.from_bf16(y)
    torch.cuda.synchronize()
    assert torch.equal(back.cpu(), x.to(torch.bfloat16).to(torch.float32))


@pytest.mark.parametrize("count", [5000, 4999])  # eight per thread; one per thread
def test_relu_and_backward(nn, count):
    g = torch.Generator().manual_seed(5)
    z = torch.randn(count, generator=g)
    da = torch.randn(count, generator=g)
    a = torch.empty(count, dtype=torch.int16, device="cuda")
    dz = torch.empty_like(a)
    nn.relu_bf16(z.cuda(), a)
    nn.relu_bf16_backward(a, da.cuda(), dz)
    torch.cuda.synchronize()
    assert torch.equal(a.cpu(), torch.relu(z).to(torch.bfloat16).view(torch.int16))
    mask = (torch.relu(z).to(torch.bfloat16).float() > 0).float()
    ref = torch.where(mask > 0, da, torch.zeros_like(da))
    assert torch.equal(dz.cpu(), ref.to(torch.bfloat16).view(torch.int16))


# w = 14: one element per thread; 12: the vector forms; 6: up2_backward's
# vector form only
@pytest.mark.parametrize("planes,h,w", [(6, 10, 14), (5, 8, 12), (3, 6, 6)])
def test_pool_and_upsample(nn, planes, h, w):
    g = torch.Generator().manual_seed(9)
    x = bf16_round(torch.randn(planes, h, w, generator=g))
    y = torch.empty(planes * (h // 2) * (w // 2), dtype=torch.int16, device="cuda")
    nn.pool2(bits(x), y, planes, h, w)
    # same FP32 order as the kernel: ((a + b) + c) + d, times 1/4, then RNE
    s = ((x[:, 0::2, 0::2] + x[:, 0::2, 1::2]) + x[:, 1::2, 0::2]) + x[:, 1::2, 1::2]
    dy = torch.randn(planes, h // 2, w // 2, generator=g)
    dx = torch.empty(planes * h * w, device="cuda")
    nn.pool2_backward(dy.cuda(), dx, planes, h, w)
    u = torch.empty(planes * 4 * h * w, dtype=torch.int16, device="cuda")
    nn.up2(bits(x), u, planes, h, w)
    du = torch.randn(planes, 2 * h, 2 * w, generator=g)
    dxu = torch.empty(planes * h * w, device="cuda")
    nn.up2_backward(du.cuda(), dxu, planes, h, w)
    torch.cuda.synchronize()
    assert torch.equal(y.cpu(), (0.25 * s).to(torch.bfloat16).view(torch.int16).reshape(-1))
    ref_dx = 0.25 * dy.repeat_interleave(2, 1).repeat_interleave(2, 2)
    assert torch.equal(dx.cpu().view(planes, h, w), ref_dx)
    ref_u = x.repeat_interleave(2, 1).repeat_interleave(2, 2)
    assert torch.equal(unbits(u).view(planes, 2 * h, 2 * w), ref_u)
    ref_du = du.view(planes, h, 2, w, 2).sum(dim=(2, 4))
    assert torch.allclose(dxu.cpu().view(planes, h, w), ref_du, rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("n", [3001, 3000])  # axpy: one, then four elements per thread
def test_adam_axpy(nn, n):
    g = torch.Generator().manual_seed(4)
    p, m, v, gr = (torch.randn(n, generator=g) for _ in range(4))
    v = v.abs()
    pd, md, vd, gd = p.cuda(), m.cuda(), v.cuda(), gr.cuda()
    pb = torch.empty(n, dtype=torch.int16, device="cuda")
    lr, b1, b2, eps, t = 1e-3, 0.9, 0.999, 1e-8, 7
    nn.adam(pd, md, vd, gd, pb, lr, t, b1, b2, eps)
    y = torch.randn(n, generator=g)
    yd = y.cuda()
    nn.axpy(-0.5, gd, yd)
    torch.cuda.synchronize()
    P, M, V, G = (q.double() for q in (p, m, v, gr))
    # the kernel takes FP32 hyperparameters: use exactly those values
    b1, b2, lr, eps = (float(np.float32(q)) for q in (b1, b2, lr, eps))
    M1 = b1 * M + (1 - b1) * G
    V1 = b2 * V + (1 - b2) * G * G
    P1 = P - lr * (M1 / (1 - b1 ** t)) / ((V1 / (1 - b2 ** t)).sqrt() + eps)
    assert np.allclose(md.cpu().double(), M1, rtol=2e-6, atol=1e-7)
    assert np.allclose(vd.cpu().double(), V1, rtol=2e-6, atol=1e-7)
    assert np.allclose(pd.cpu().double(), P1, rtol=2e-6, atol=1e-6)
    assert torch.equal(pb.cpu(), pd.cpu().to(torch.bfloat16).view(torch.int16))
    assert np.allclose(yd.cpu().double(), y.double() - 0.5 * G, rtol=1e-6, atol=1e-7)


@pytest.mark.parametrize("c,hw", [(24, 49), (40, 128)])  # one-pass and 64-pixel-row forms of the head
def test_head_and_loss(nn, c, hw):
    g = torch.Generator().manual_seed(12)
    n = 5
    a = bf16_round(torch.relu(torch.randn(c, n, hw, generator=g)))
    wl = torch.randn(c, generator=g)
    bl = torch.randn(1, generator=g)
    out = torch.empty(n, device="cuda")
    nn.gap_linear(bits(a), wl.cuda(), bl.cuda(), out, n, c, hw)
    dout = torch.randn(n, generator=g)
    da = torch.empty(c * n * hw, device="cuda")
    dwl = torch.empty(c, device="cuda")
    dbl = torch.empty(1, device="cuda")
    nn.gap_linear_backward(bits(a), wl.cuda(), dout.cuda(), da, dwl, dbl, n, c, hw)
    pred = torch.randn(1000, generator=g)
    tgt = torch.randn(1000, generator=g)
    grad = torch.empty(1000, device="cuda")
    work = torch.empty(nn.mse_work(1000), dtype=torch.float64, device="cuda")
    ssq = torch.empty(1, dtype=torch.float64, device="cuda")
    nn.mse(pred.cuda(), tgt.cuda(), 0.25, grad, work, ssq)
    torch.cuda.synchronize()
    A = a.double()
    ref = (A.mean(dim=2) * wl.double()[:, None]).sum(0) + bl.double()
    assert np.allclose(out.cpu().double(), ref, rtol=1e-5, atol=1e-6)
    ref_da = dout.double()[None, :, None] * wl.double()[:, None, None] / hw * torch.ones(c, n, hw, dtype=torch.float64)
    assert np.allclose(da.cpu().double().view(c, n, hw), ref_da, rtol=1e-6, atol=1e-7)
    assert np.allclose(dwl.cpu().double(), (A.mean(dim=2) * dout.double()[None, :]).sum(1), rtol=1e-5, atol=1e-6)
    assert abs(dbl.item() - dout.double().sum().item()) <= 1e-5
    d = (pred - tgt).double()  # the kernel forms the difference in FP32, the sum in FP64
    want = float((d * d).sum())
    assert abs(ssq.item() - want) <= 1e-12 * want
    assert np.allclose(grad.cpu().double(), 0.5 * d, rtol=1e-6, atol=1e-7)


def test_invalid_sizes_rejected(nn):
    x = torch.zeros(16, dtype=torch.int16, device="cuda")
    z = torch.zeros(16, device="cuda")
    with pytest.raises(Exception, match="EINVAL"):
        nn.conv3x3(x, x, None, 0, 1, 1, 4, 4, z=z)
    with pytest.raises(Exception, match="EINVAL"):
        nn.conv3x3(x, x, None, 1, 1, 1, 4, 4)  # neither output
    with pytest.raises(Exception, match="EINVAL"):
        nn.pool2(x, x, 1, 3, 4)  # odd side


# ---- the assembled U-Net against a torch CPU model of the same arithmetic ----

class _STRound(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x):
        return x.to(torch.bfloat16).to(torch.float32)

    @staticmethod
    def backward(ctx, g):
        return g


def ref_unet(nn, net, p, rho):
    """Forward of the U-Net with parameters p (CPU FP32 leaf), on rho (CPU [n][s][s])."""
    ch, plan = net.ch, net.plan
    L = len(ch)
    rnd = _STRound.apply

    def W(i):
        cin, cout, _ = plan[i]
        ow, ob = net.offs[i]
        return rnd(p[ow:ob]).view(cout, 3, 3, cin).permute(0, 3, 1, 2), p[ob:ob + cout]

    def conv(x, i, relu=True):
        w, b = W(i)
        z = Fn.conv2d(x, w, b, padding=1)
        return rnd(torch.relu(z)) if relu else z

    x = rnd(rho.unsqueeze(1))
    skips, li = [], 0
    for l in range(L):
        x = conv(conv(x, li), li + 1)
        li += 2
        skips.append(x)
        if l < L - 1:
            x = rnd(Fn.avg_pool2d(x, 2))
    bottom = x
    lo = net.lin_off
    F = (bottom.mean(dim=(2, 3)) * p[lo:lo + ch[-1]]).sum(1) + p[lo + ch[-1]]
    y = bottom
    for l in range(L - 2, -1, -1):
        y = torch.cat([y.repeat_interleave(2, 2).repeat_interleave(2, 3), skips[l]], dim=1)
        y = conv(conv(y, li), li + 1)
        li += 2
    S = conv(y, li, relu=False)[:, 0]
    return F, S


@pytest.mark.parametrize("side,batch", [(32, 3), (64, 2)])
def test_unet_forward_backward_matches_cpu_model(nn, side, batch):
    g = torch.Generator().manual_seed(side)
    net = nn.UNet(side, batch, seed=side)
    rho = torch.rand(batch, side, side, generator=g)
    Ft = torch.randn(batch, generator=g)
    St = torch.randn(batch, side, side, generator=g) * 0.1
    F, S = net.forward(rho.cuda())
    dF, dS = net.loss_grad(Ft.cuda(), St.cuda(), wF=1.0, wS=2.0)
    net.backward(dF, dS)
    torch.cuda.synchronize()
    p = net.p.cpu().clone().requires_grad_()
    Fr, Sr = ref_unet(nn, net, p, rho)
    loss = ((Fr - Ft) ** 2).mean() + 2.0 * ((Sr - St) ** 2).mean()
    loss.backward()
    assert rel(F.cpu(), Fr.detach()) < 2e-2
    assert rel(S.cpu(), Sr.detach()) < 2e-2
    lsum = net.loss.cpu().double()
    lgpu = lsum[0].item() / batch + 2.0 * lsum[1].item() / (batch * side * side)
    assert abs(lgpu - loss.item()) <= 2e-2 * loss.item()
    gg, gr = net.g.cpu(), p.grad
    for i, (ow, ob) in enumerate(net.offs):
        cout = net.plan[i][1]
        a, b = gg[ow:ob + cout], gr[ow:ob + cout]
        cos = float((a.double() @ b.double()) / (a.double().norm() * b.double().norm() + 1e-30))
        assert cos > 0.995 and rel(a, b) < 0.1, (i, cos, rel(a, b))
    lo = net.lin_off
    assert rel(gg[lo:], gr[lo:]) < 2e-2


def test_unet_overfits_small_set(nn):
    """A few hundred Adam steps drive the training loss on 4 samples down by 20x."""
    g = torch.Generator().manual_seed(1)
    side, batch = 32, 4
    net = nn.UNet(side, batch, seed=3)
    rho = torch.rand(batch, side, side, generator=g).cuda()
    yy, xx = torch.meshgrid(torch.linspace(-1, 1, side), torch.linspace(-1, 1, side), indexing="ij")
    St = torch.stack([torch.exp(-(xx ** 2 + yy ** 2) * (k + 1)) for k in range(batch)]).cuda()
    Ft = torch.tensor([0.5, -0.25, 1.0, 0.0]).cuda()
    first = None
    for it in range(300):
        net.forward(rho)
        dF, dS = net.loss_grad(Ft, St)
        net.backward(dF, dS)
        net.step(2e-3)
        if it == 0:
            torch.cuda.synchronize()
            first = net.loss.cpu().clone()
    torch.cuda.synchronize()
    last = net.loss.cpu()
    l0 = first[0] / batch + first[1] / St.numel()
    l1 = last[0] / batch + last[1] / St.numel()
    assert torch.isfinite(last).all()
    assert l1 < l0 / 20, (l0.item(), l1.item())
