"""The HBM streaming probe (gs_fluid_stream_probe), whose rates are the
ceilings the stage kernels are compared with, computes what it claims: c = a
and c = a + b, bit for bit, for sizes with and without a partial last
block, with and without non-temporal stores."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [2, 2048, 2 * 1000003])
@pytest.mark.parametrize("nt", [False, True])
def test_stream_probe_copies_and_adds(n, nt):
    import torch
    from paper_1812_07977_amd import stream_probe
    print(f"case: stream probe n={n} nontemporal={nt}", flush=True)
    g = torch.Generator(device="cpu").manual_seed(n)
    a = torch.randn(n, dtype=torch.float64, generator=g).cuda()
    b = torch.randn(n, dtype=torch.float64, generator=g).cuda()
    c = torch.full_like(a, float("nan"))
    stream_probe(a, c, nontemporal=nt)
    torch.cuda.synchronize()
    assert torch.equal(c, a)
    c.fill_(float("nan"))
    stream_probe(a, c, b=b, nontemporal=nt)
    torch.cuda.synchronize()
    assert torch.equal(c, a + b)
