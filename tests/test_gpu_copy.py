"""The library's streaming device copy (the bandwidth reference of the
measurement) copies exactly, for whole-wave, ragged and tiny sizes."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nbytes,offset", [(16, 0), (4096 + 48, 16), ((64 << 20) + 16 * 12345, 32), (0, 0)])
def test_copy_device_is_exact(nbytes, offset):
    import torch
    import paper_1503_01405_amd as P
    print(f"case: copy {nbytes} bytes at offset {offset}", flush=True)
    g = torch.Generator(device="cpu").manual_seed(nbytes)
    host = torch.randint(0, 256, (nbytes + offset + 64,), dtype=torch.uint8, generator=g)
    src = host.to("cuda")
    dst = torch.zeros_like(src)
    P.pond_copy_device(dst[offset:].data_ptr(), src[offset:].data_ptr(), nbytes)
    torch.cuda.synchronize()
    out = dst.cpu()
    assert torch.equal(out[offset:offset + nbytes], host[offset:offset + nbytes])
    assert int(out[:offset].sum()) == 0 and int(out[offset + nbytes:].sum()) == 0
    with pytest.raises(P.PondError):
        P.pond_copy_device(dst[offset + 8:].data_ptr(), src[offset:].data_ptr(), 16)
