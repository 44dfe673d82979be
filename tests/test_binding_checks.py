"""Host-side argument checks of the Python binding (no GPU needed): buffers handed to
the library as raw pointers must have the exact shape, dtype and layout the C ABI
writes, and propagators must be complex [n_t, Lz, Ly, Lx, 12, 12]."""
import pytest

torch = pytest.importorskip("torch")

import paper_1510_00903_amd as bbc


def test_check_tensor_accepts_exact_buffer():
    t = torch.zeros((2, 3, 4, 16), dtype=torch.complex128)
    bbc._check_tensor(t, (2, 3, 4, 16), torch.complex128, "out", host_ok=True)


@pytest.mark.parametrize("t,why", [
    (torch.zeros((2, 3, 4, 8), dtype=torch.complex128), "shape"),
    (torch.zeros((2, 3, 4, 16), dtype=torch.complex64), "dtype"),
    (torch.zeros((2, 3, 16, 4), dtype=torch.complex128).transpose(-1, -2), "contiguous"),
    ([0.0] * 16, "torch tensor"),
])
def test_check_tensor_rejects(t, why):
    with pytest.raises(bbc.BBCError, match=why):
        bbc._check_tensor(t, (2, 3, 4, 16), torch.complex128, "out", host_ok=True)


def test_check_tensor_host_only_when_allowed():
    t = torch.zeros((1, 16), dtype=torch.complex128)
    with pytest.raises(bbc.BBCError, match="device"):
        bbc._check_tensor(t, (1, 16), torch.complex128, "scale")


def test_prop_dtype():
    z = torch.zeros((1, 2, 2, 2, 12, 12), dtype=torch.complex64)
    assert bbc._prop_dtype(z, "S") == bbc.F32
    assert bbc._prop_dtype(z.to(torch.complex128), "S") == bbc.F64
    with pytest.raises(bbc.BBCError):
        bbc._prop_dtype(z.real, "S")
    with pytest.raises(bbc.BBCError):
        bbc._prop_dtype(torch.zeros((2, 2, 2, 12, 12), dtype=torch.complex64), "S")
