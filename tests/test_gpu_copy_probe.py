"""The library's streaming copy (the bandwidth ceiling of the benchmark)
copies every element, for sizes below, at and above one workgroup's and one
grid's worth of elements."""

import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(autouse=True, scope="module")
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")


@pytest.mark.parametrize("n", [1, 1023, 1024, 1025, 16384 * 1024 + 7, 3 * 16384 * 1024 + 5])
def test_copy_probe_copies_every_element(n):
    import paper_1402_3545_amd as G
    src = torch.randn(n, dtype=torch.float64, device="cuda")
    out = torch.full_like(src, -7.0)
    G.gmg_copy_probe(src, out)
    torch.cuda.synchronize()
    assert torch.equal(out, src)


def test_copy_probe_of_zero_bytes_is_a_no_op():
    import paper_1402_3545_amd as G
    a = torch.ones(4, dtype=torch.float64, device="cuda")
    b = torch.zeros(4, dtype=torch.float64, device="cuda")
    assert G._lib.gmg_copy_probe(a.data_ptr(), b.data_ptr(), 0, None) == 0
    G.gmg_copy_probe(a[:0], b[:0])
    torch.cuda.synchronize()
    assert torch.equal(b, torch.zeros_like(b))
