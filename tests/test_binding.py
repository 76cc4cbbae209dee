"""The Python binding refuses tensors whose dtype, device, size or layout would
let the library read or write past a buffer (checked on the host, before any
library call)."""
import pytest

torch = pytest.importorskip("torch")

from paper_1310_4374_amd import api  # noqa: E402

CPU = torch.device("cpu")


def test_vec_accepts_matching_float64_and_rejects_the_rest():
    t = torch.zeros(5, dtype=torch.float64)
    assert api._vec(t, 5, CPU, "q").data_ptr() == t.data_ptr()
    with pytest.raises(ValueError, match="float64"):
        api._vec(torch.zeros(5, dtype=torch.float32), 5, CPU, "q")
    with pytest.raises(ValueError, match="5 elements"):
        api._vec(torch.zeros(4, dtype=torch.float64), 5, CPU, "q")
    with pytest.raises(ValueError, match="float64 on"):
        api._vec(t, 5, torch.device("meta"), "q")
    with pytest.raises(TypeError):
        api._vec([0.0] * 5, 5, CPU, "q")


def test_field_outputs_must_be_contiguous_3_by_n():
    assert api._field_out(torch.zeros(3, 7, dtype=torch.float64), 7, CPU, "field") is not None
    with pytest.raises(ValueError):
        api._field_out(torch.zeros(7, 3, dtype=torch.float64).t(), 7, CPU, "field")
    with pytest.raises(ValueError):
        api._field_out(torch.zeros(3, 6, dtype=torch.float64), 7, CPU, "field")
    with pytest.raises(ValueError):
        api._field_out(torch.zeros(3, 7, dtype=torch.float32), 7, CPU, "field")


def test_offsets_must_cover_the_particles():
    api._check_offsets([0, 3, 10], 10)
    for bad in ([1, 3, 10], [0, 3, 9], [0, 3, 3, 10], [0]):
        with pytest.raises(ValueError):
            api._check_offsets(bad, 10)


def test_positions_must_be_3_by_n_float64():
    x = torch.zeros(3, 9, dtype=torch.float64)
    assert api._soa(x, CPU).shape == (3, 9)
    assert api._soa(torch.zeros(9, 3, dtype=torch.float64), CPU).shape == (3, 9)
    with pytest.raises(ValueError):
        api._soa(torch.zeros(4, 9, dtype=torch.float64), CPU)
    with pytest.raises(ValueError):
        api._soa(torch.zeros(3, 9, dtype=torch.float32), CPU)
