"""The device probe that the benchmark's roofline reports beside the
published peaks (FP64 matrix cores and FMAs 78.6 TFLOP/s, HBM 8 TB/s on the
MI355X): the measured rates are positive and in the range that hardware can
deliver, and the device is the 256-CU part the rooflines assume."""
import pytest

from gpu_util import announce

pytestmark = pytest.mark.gpu


def test_probe_peaks_in_range():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_2002_00322_amd as pa
    announce("probe peaks, 256 MiB copy")
    pk = pa.probe_peaks(256 << 20)
    announce(f"peaks {pk}")
    assert pk["compute_units"] == 256
    # no loop may beat the published rate (78.6 TFLOP/s at the 2.4 GHz peak clock)
    assert 20.0 < pk["fp64_mfma_tflops"] < 1.05 * 78.6
    assert 20.0 < pk["fp64_fma_tflops"] < 1.05 * 78.6
    assert 1.0 < pk["copy_tbps"] < 8.0
