"""Device-ceiling measurement entry point (used for the roofline fractions)."""
import pytest

pytestmark = pytest.mark.gpu


def test_measured_peaks_are_plausible_and_sizes_checked():
    import torch
    import paper_2609_09990_amd as pk
    f, c = pk.measure_peaks(1 << 28)
    print(f"fp64 MFMA {f:.1f} TFLOP/s, copy {c:.0f} GB/s", flush=True)
    # published MI355X figures: 78.6 TFLOP/s fp64 matrix, 8 TB/s HBM
    assert 20.0 < f < 90.0
    assert 500.0 < c < 9000.0
    a = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    import ctypes as C
    f_, c_ = C.c_double(), C.c_double()
    code = pk.dmrg_measure_peaks(None, C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()), 1 << 20,
                                 C.byref(f_), C.byref(c_))
    assert code == -1 and "4 MiB" in pk.dmrg_last_error().decode()
