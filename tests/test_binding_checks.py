"""The binding refuses tensors of the wrong dtype, shape, size, layout or place before anything
reaches the library (no GPU needed: every check below fires ahead of the device check, and a
well-formed host tensor is refused as not on the device)."""
import pytest

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    from paper_2501_08261_amd import lib
    return lib


def test_dtype_shape_numel(lib):
    x = torch.zeros((4, 16), dtype=torch.float64)
    with pytest.raises(ValueError, match="dtype"):
        lib._ptr(x.float(), "params", torch.float64, shape=(None, 16))
    with pytest.raises(ValueError, match="shape"):
        lib._ptr(torch.zeros((4, 15), dtype=torch.float64), "params", torch.float64, shape=(None, 16))
    with pytest.raises(ValueError, match="shape"):
        lib._ptr(torch.zeros(64, dtype=torch.float64), "params", torch.float64, shape=(None, 16))
    with pytest.raises(ValueError, match="elements"):
        lib._ptr(torch.zeros((2, 3, 99), dtype=torch.float32), "out", torch.float32, numel=2 * 3 * 100)
    with pytest.raises(ValueError, match="contiguous"):
        lib._ptr(torch.zeros((16, 4), dtype=torch.float64).t(), "params", torch.float64, shape=(None, 16))
    with pytest.raises(ValueError, match="device tensor"):
        lib._ptr(x, "params", torch.float64, shape=(None, 16))
    with pytest.raises(ValueError, match="torch tensor"):
        lib._ptr([0.0] * 16, "params")
    assert lib._ptr(None, "status", torch.int32, numel=4) is None


def test_psd_layout(lib):
    n = 64
    with pytest.raises(ValueError, match="shape"):
        lib._psd_struct(torch.zeros((3, n // 2), dtype=torch.float64), n, 3e-4, 0.02)
    with pytest.raises(ValueError, match="dtype"):
        lib._psd_struct(torch.zeros((3, n // 2 + 1), dtype=torch.float32), n, 3e-4, 0.02)
    with pytest.raises(ValueError, match="device tensor"):          # a host PSD never becomes a kernel pointer
        lib._psd_struct(torch.zeros((3, n // 2 + 1), dtype=torch.float64), n, 3e-4, 0.02)


def test_real_dtype_follows_precision(lib):
    assert lib.real_dtype(lib.LT_FP64) == torch.float64
    assert lib.real_dtype(lib.LT_MIXED) == torch.float32
