"""The bandwidth probe pic_copy_probe (measurement only) through the C ABI:
every array copied word for word, ragged sizes, argument checks."""
import ctypes as C

import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pic():
    from paper_0808_4078_amd import pic as p
    p.lib()
    return p


@pytest.mark.parametrize("narrays,words,chunk", [(1, 1, 256), (3, 1000003, 256), (7, 4097, 1024),
                                                 (8, 65536 * 257 + 5, 32768), (2, 100, 4096)])
def test_copy_probe_copies_every_word(pic, narrays, words, chunk):
    import torch
    g = torch.Generator(device="cuda").manual_seed(narrays)
    src = [torch.randint(-2 ** 31, 2 ** 31 - 1, (words,), dtype=torch.int32, device="cuda", generator=g)
           for _ in range(narrays)]
    dst = [torch.zeros_like(t) for t in src]
    pic.copy_probe(src, dst, chunk=chunk)
    torch.cuda.synchronize()
    assert all(bool(torch.equal(a, b)) for a, b in zip(src, dst))


def test_copy_probe_rejects_bad_arguments(pic):
    import torch
    a = torch.zeros(16, dtype=torch.int32, device="cuda")
    b = torch.zeros(16, dtype=torch.int32, device="cuda")
    arr_a = (C.c_void_p * 9)(*([a.data_ptr()] * 9))
    arr_b = (C.c_void_p * 9)(*([b.data_ptr()] * 9))
    L = pic.lib()
    assert L.pic_copy_probe(arr_a, arr_b, 0, 16, 256, None) == pic.PIC_E_INVALID_ARG
    assert L.pic_copy_probe(arr_a, arr_b, 9, 16, 256, None) == pic.PIC_E_INVALID_ARG
    assert L.pic_copy_probe(arr_a, arr_b, 1, -1, 256, None) == pic.PIC_E_INVALID_ARG
    assert L.pic_copy_probe(arr_a, arr_b, 1, 16, 100, None) == pic.PIC_E_INVALID_ARG
    assert L.pic_copy_probe(arr_a, arr_b, 1, 16, 0, None) == pic.PIC_E_INVALID_ARG
    assert L.pic_copy_probe(None, arr_b, 1, 16, 256, None) == pic.PIC_E_INVALID_ARG
    nul = (C.c_void_p * 1)(None)
    assert L.pic_copy_probe(nul, arr_b, 1, 16, 256, None) == pic.PIC_E_INVALID_ARG
    assert L.pic_copy_probe(arr_a, arr_b, 1, 0, 256, None) == 0
    with pytest.raises(ValueError):
        pic.copy_probe([a], [torch.zeros(8, dtype=torch.int32, device="cuda")])
