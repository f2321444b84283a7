"""The streaming probe behind the measured bandwidth ceiling: its copy and
write launches store exactly what they should, over every grid size the
ceiling sweep uses and a length that leaves a ragged last round."""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("nt", [False, True])
def test_probe_copy_and_write(nt):
    from paper_2111_00847_amd import api
    n = (3 << 20) + 48                      # bytes: 16-byte elements, not a multiple of any grid's stride
    src = torch.randint(0, 2**31 - 1, (n // 4,), dtype=torch.int32, device="cuda")
    for blocks in (256, 4096, 16384):
        dst = torch.zeros_like(src)
        api.lbm_bandwidth_probe(2, dst, src, n, blocks, nt)
        torch.cuda.synchronize()
        assert torch.equal(dst, src), blocks
        api.lbm_bandwidth_probe(1, dst, None, n, blocks, nt)
        torch.cuda.synchronize()
        v = 0x9E3779B9
        want = torch.tensor([v, v + 1, v + 2, v + 3], dtype=torch.int64).to(torch.uint32).view(torch.int32)
        assert torch.equal(dst.view(-1, 4).cpu(), want.expand(n // 16, 4)), blocks
        sink = torch.zeros(blocks * 256, dtype=torch.int32, device="cuda")
        api.lbm_bandwidth_probe(0, sink, src, n, blocks, nt)
        torch.cuda.synchronize()
        x = src.view(-1, 4).cpu().numpy().astype("uint32")
        folded = x[:, 0] ^ x[:, 1] ^ x[:, 2] ^ x[:, 3]
        import numpy as np
        assert int(np.bitwise_xor.reduce(sink.cpu().numpy().astype("uint32"))) == int(np.bitwise_xor.reduce(folded))
