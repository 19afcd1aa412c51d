"""Host-side contract of bench.py: the product runs on one GPU, so a request
for more ranks ends before any device or library call, with a message and a
nonzero status."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(args, env_extra=None):
    env = dict(os.environ)
    env.update(env_extra or {})
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + args, cwd=ROOT, env=env,
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_refused():
    r = _run(["--gpus", "2"])
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_world_size_above_one_refused():
    r = _run(["--gpus", "1"], {"WORLD_SIZE": "4"})
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def _roofline(names, dom, flops, nbytes, ms, launches):
    sys.path.insert(0, ROOT)
    import bench
    n = len(names)
    r = {"t_k": [0.0] * n, "l_k": [0] * n,
         "cnt": {"launches_kernel": [0] * n, "flops_kernel": [0.0] * n, "bytes_kernel": [0.0] * n,
                 "units_kernel": [0.0] * n}}
    r["t_k"][dom], r["l_k"][dom] = ms, launches
    r["cnt"]["launches_kernel"][dom] = launches
    r["cnt"]["flops_kernel"][dom] = flops
    r["cnt"]["bytes_kernel"][dom] = nbytes
    return bench.roofline(names, r, 1, "grid32")


def test_roofline_bound_of_each_kernel_family():
    """The dominant kernel's roofline: the GEMM against the HBM peak (bytes),
    the QR, SVD (including the narrow first pass, whose combined entry starts
    with its own name) and Cholesky kernels against the FP64 peak (flops),
    each from the algorithmic figure per launch over the average launch time."""
    names = ["gemm_kernel<double>", "qr_kernel<128, 512, 64>",
             "svd_narrow_kernel<128, 512, 64> + svd_kernel<128, 512>", "chol_kernel"]
    for dom, bound in ((0, "hbm"), (1, "alu"), (2, "alu"), (3, "alu")):
        roof = _roofline(names, dom, flops=4e12, nbytes=8e9, ms=10.0, launches=4)
        assert roof["bound"] == bound, names[dom]
        assert roof["kernel"] == names[dom]
        if bound == "hbm":
            assert abs(roof["achieved"] - 8e9 / 4 / 2.5e-3 / 1e9) < 1e-6  # GB/s per launch
            assert abs(roof["frac"] - roof["achieved"] / 8000.0) < 1e-12
        else:
            assert abs(roof["achieved"] - 4e12 / 4 / 2.5e-3 / 1e12) < 1e-9  # TFLOP/s per launch
            assert abs(roof["frac"] - roof["achieved"] / 78.6) < 1e-12
