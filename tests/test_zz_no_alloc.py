"""The allocation-free weight gradient (fdtd_nn_conv3x3_wgrad_noalloc, for
callers that cannot allocate device memory) against the workspace entry
point fdtd_nn_conv3x3_wgrad through the C ABI: the same dw and db bit for bit
(same kernels and split plan) on calls in a row, each smaller than the one
before, so the library's static scratch holds the previous call's partial
sums when the next one starts; and EINVAL, with nothing launched, for a
layer whose workspace exceeds the static array."""
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nn():
    from paper_2203_01462_amd import nn as m
    m.load_library()
    torch.cuda.set_device(0)
    return m


def bf16_bits(nn, count, gen):
    x = torch.randn(count, generator=gen).cuda()
    return nn.to_bf16(x)


# (n, cin, cout, h, w): the deepest surrogate layer at batch 32 (largest
# workspace of the plan), a smaller tiled layer, then the generic kernel
CASES = [(32, 256, 256, 16, 16), (4, 64, 96, 24, 48), (3, 3, 5, 40, 40)]


def test_noalloc_matches_workspace_entry_point(nn):
    gen = torch.Generator().manual_seed(5)
    for n, cin, cout, h, w in CASES:
        work_floats = nn.wgrad_work(n, cin, cout, h, w)
        assert work_floats <= 16 << 20
        x = bf16_bits(nn, cin * n * h * w, gen)
        dz = bf16_bits(nn, cout * n * h * w, gen)
        dw_ref = torch.empty(cout * cin * 9, device="cuda")
        db_ref = torch.empty(cout, device="cuda")
        work = torch.empty(work_floats, device="cuda")
        nn.conv3x3_wgrad(x, dz, dw_ref, db_ref, work, n, cin, cout, h, w)
        dw = torch.full((cout * cin * 9,), float("nan"), device="cuda")
        db = torch.full((cout,), float("nan"), device="cuda")
        nn.conv3x3_wgrad_noalloc(x, dz, dw, db, n, cin, cout, h, w)
        torch.cuda.synchronize()
        print(f"[no-alloc] n={n} cin={cin} cout={cout} {h}x{w}: workspace {work_floats} floats, "
              f"max|dw - ref| = {(dw - dw_ref).abs().max().item():.3e}", flush=True)
        assert torch.equal(dw, dw_ref) and torch.equal(db, db_ref)


def test_noalloc_rejects_a_layer_beyond_the_scratch(nn):
    from paper_2203_01462_amd.fdtd import FDTDError
    n, cin, cout, h, w = 1, 2048, 1024, 16, 16
    assert nn.wgrad_work(n, cin, cout, h, w) > 16 << 20
    x = torch.zeros(cin * n * h * w, dtype=torch.int16, device="cuda")
    dz = torch.zeros(cout * n * h * w, dtype=torch.int16, device="cuda")
    dw = torch.full((cout * cin * 9,), 7.0, device="cuda")
    db = torch.full((cout,), 7.0, device="cuda")
    with pytest.raises(FDTDError) as e:
        nn.conv3x3_wgrad_noalloc(x, dz, dw, db, n, cin, cout, h, w)
    torch.cuda.synchronize()
    assert e.value.name == "EINVAL" and "scratch" in str(e.value)
    assert torch.all(dw == 7.0) and torch.all(db == 7.0)  # nothing ran
