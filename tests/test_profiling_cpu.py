"""The rocprofv3 summary helpers on the CPU: kernel names to families (the
per-kernel tables and the HBM-traffic summary group launches by family)."""
import pytest

from paper_2205_07805_amd import profiling as P


@pytest.mark.parametrize("name,fam", [
    ("void igs::opreduce_kernel<8, double, true>(igs::Work, long long, int)", "opreduce"),
    ("void igs::reduce_kernel<8, true, true, double>(igs::Work, long long, int)", "reduce"),
    ("void igs::update_kernel<true, true, double, 8>(igs::Work, long long, int)", "update"),
    ("void igs::xupdate_kernel<double, 8>(igs::Work, long long, double*)", "xupdate"),
    ("void igs::xupdate_kernel<float, 0>(igs::Work, long long, double*)", "xupdate"),
    ("igs::coef_kernel(igs::Work, int, int)", "coef"),
    ("igs::lsq_kernel(igs::Work, int, int)", "lsq"),
    ("void igs::spmv_ell_kernel<7, 2, double, double>(long long)", "spmv"),
    ("void igs::spmv_csr_kernel<8, 4, double, double>(long long)", "spmv"),
    ("igs::gemv_dense_kernel(long long, double const*)", "spmv"),
    ("__amd_rocclr_copyBuffer", None),
])
def test_kernel_families(name, fam):
    assert P.family(name) == fam
