"""Each device kernel against host evaluations of its definition (through the
h2_selftest diagnostic entry point)."""
import pytest

pytestmark = pytest.mark.gpu

NAMES = ["gemm_f64_nn", "gemm_f64_tn", "gemm_f64_nt", "gemm_f64_tt",
         "gemm_f32_nn", "gemm_f32_tn", "gemm_f32_nt", "gemm_f32_tt",
         "qr_w20", "qr_w64", "qr_w128", "qr_split_w100", "qr_split_w48", "svd_w24", "svd_w64", "svd_w128", "svd_qrcp_w40", "svd_qrcp_w128", "svd_qrcp_w100_r20",
         "chol_w12", "chol_w32", "chol_w50", "svd_empty",
         "svd_qrcp_w100_r20_x1024", "svd_qrcp_w128_x1024", "svd_w128_x1024",
         "gemm_f64_nt_kdev", "gemm_f32_tn_kdev", "qr_w50_m300", "qr_w32_m129"]
TOL = [1e-14] * 4 + [3e-6] * 4 + [1e-13] * 5 + [1e-9] * 3 + [1e-12] * 3 + [1e-12] * 3 + [0.0] + [1e-12, 1e-12, 1e-9] \
    + [1e-14, 3e-6] + [1e-13] * 2


def test_kernel_selftest():
    from paper_2403_01566_amd import h2
    ctx = h2.Context(0)
    err = h2.selftest(ctx)
    print(dict(zip(NAMES, err)), flush=True)
    assert len(err) == len(NAMES)
    bad = {n: e for n, e, t in zip(NAMES, err, TOL) if not (e <= t)}
    assert not bad, bad
