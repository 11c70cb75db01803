"""Host-side argument checks of the Python binding: buffers the kernels would read or
write past their end, or in a type they do not handle, are refused with a ValueError
before any call crosses the C ABI (no GPU needed)."""
import numpy as np
import pytest
import torch

from paper_1908_06742_amd import _lib as L
from paper_1908_06742_amd.batch import Batch
from paper_1908_06742_amd.lattice import Lattice, check_extract_out, output_mask

CPU = torch.device("cpu")


def _host_lattice(nx=8, ny=4):
    """A Lattice object with no handle: its methods run their checks, and a call that
    passed them would fail at the (NULL) handle."""
    lat = Lattice.__new__(Lattice)
    lat.nx, lat.ny, lat.device, lat.stream, lat._h = nx, ny, CPU, None, None
    return lat


def test_output_mask_and_unknown_names():
    assert output_mask(["rho"]) == 1 and output_mask(["wz"]) == 1 << 7
    assert output_mask(L.OUTPUTS) == (1 << len(L.OUTPUTS)) - 1
    with pytest.raises(ValueError, match="unknown output"):
        output_mask(["vorticity"])


@pytest.mark.parametrize("dtype", [torch.float16, torch.bfloat16, torch.int32])
def test_extract_refuses_output_types_the_kernels_do_not_write(dtype):
    with pytest.raises(ValueError, match="float64 or float32"):
        _host_lattice().extract(["ux"], dtype=dtype)
    with pytest.raises(ValueError, match="float64 or float32"):
        _host_lattice().extract(["ux"], out=torch.empty((16, 4, 8), dtype=dtype))


def test_extract_refuses_a_buffer_without_the_highest_selected_plane():
    # wz is plane 7: the kernel writes out[7 * ny * nx + c], so 8 planes are needed
    with pytest.raises(ValueError, match="8 planes"):
        _host_lattice().extract(["wz"], out=torch.empty((4, 4, 8), dtype=torch.float32))
    with pytest.raises(ValueError, match="8 planes"):
        check_extract_out(torch.empty(8 * 32 - 1, dtype=torch.float64), output_mask(["wz"]), 4, 8, CPU)
    assert check_extract_out(torch.empty(8 * 32, dtype=torch.float64), output_mask(["wz"]), 4, 8, CPU) == 0
    assert check_extract_out(torch.empty((4, 4, 8), dtype=torch.float32), output_mask(["phi"]), 4, 8, CPU) == 1


def test_extract_refuses_non_contiguous_or_foreign_buffers():
    strided = torch.empty((16, 8, 4), dtype=torch.float32).transpose(1, 2)
    with pytest.raises(ValueError, match="contiguous"):
        _host_lattice().extract(["ux"], out=strided)
    with pytest.raises(ValueError, match="is on"):
        check_extract_out(torch.empty((16, 4, 8)), 1, 4, 8, torch.device("cuda", 0))
    with pytest.raises(ValueError, match="torch tensor"):
        check_extract_out(np.empty((16, 4, 8), np.float32), 1, 4, 8, CPU)


def test_set_populations_and_init_refuse_wrong_shapes():
    lat = _host_lattice()
    with pytest.raises(ValueError, match=r"\(9, 4, 8\)"):
        lat.set_populations(np.zeros((9, 8, 4)), np.zeros((9, 4, 8)))
    with pytest.raises(ValueError, match=r"\(9, 4, 8\)"):
        lat.set_populations(np.zeros((9, 4, 8)), np.zeros((8, 4, 8)))
    with pytest.raises(ValueError, match="does not broadcast"):
        lat.init(np.ones((4, 7)), 0.0, 0.0, 1.0)


def test_batch_refuses_fields_and_output_types_of_the_wrong_size():
    class P:
        nx, ny = 8, 4
    b = Batch.__new__(Batch)
    b.problems, b.n, b.device, b.stream, b._h, b.total_nodes = [P(), P()], 2, CPU, None, None, 64
    z = torch.zeros(63, dtype=torch.float64)
    with pytest.raises(ValueError, match="64 elements"):
        b.init_device(z, z, z, z)
    with pytest.raises(ValueError, match="32 elements"):
        b.init_instance(1, torch.zeros((4, 7), dtype=torch.float64), 0.0, 0.0, 1.0)
    with pytest.raises(ValueError, match="float64 or float32"):
        b.extract(0, ["ux"], dtype=torch.float16)
