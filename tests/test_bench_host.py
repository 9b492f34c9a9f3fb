"""Host logic of bench.py (no GPU): the rocprofv3 counter summary and the
traffic lookup that the roofline line reports."""
import csv
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402

FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def write_csv(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for i, (name, v) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": v})


def test_counter_summary_calibrates_and_round_trips(tmp_path):
    spmv = "void gfem::(anonymous namespace)::k_pcg_spmv_p<float, 256>(gfem::MatView, int)"
    red = "void at::native::reduce_kernel<512, 1>(at::native::ReduceOp<float>)"
    fetch = tmp_path / "f.csv"
    wr = tmp_path / "w.csv"
    # calibration: the 64 MiB sum reads FETCH 32768 KiB (factor 2); the copy writes 65536 KiB (factor 1)
    write_csv(fetch, "FETCH_SIZE", [(red, 32768.0), (spmv, 30000.0), (spmv, 32000.0), ("__amd_rocclr_copyBuffer", 10.0)])
    write_csv(wr, "WRITE_SIZE", [("__amd_rocclr_copyBuffer", 65536.0), (spmv, 1000.0), (spmv, 3000.0)])
    out = tmp_path / "counters.txt"
    bench.write_counter_summary(str(fetch), str(wr), 64, "cmd F", "cmd W", out_path=str(out))
    text = out.read_text()
    assert "calib_read_factor 2.0000" in text and "calib_write_factor 1.0000" in text
    expect = (2.0 * 31000.0 + 1.0 * 2000.0) * 1024.0
    assert bench.measured_traffic(str(out)) == pytest.approx(expect)
    assert "k_pcg_spmv_p<float, 256>" in text
    # a summary taken from other kernel sources is not reported
    out.write_text(text.replace(text.split("kernel_sources_sha256 ")[1].split()[0], "0" * 64))
    assert bench.measured_traffic(str(out)) is None


def test_kernel_short_name():
    assert bench.kernel_short_name("void gfem::(anonymous namespace)::k_pcg_gpass<float, false, 256>(int, a)") == \
        "k_pcg_gpass<float, false, 256>"
    assert bench.kernel_short_name("void gfem::k_damage(int, int const*)") == "k_damage"


def test_pulled_block_inputs():
    """The quasi-static blocks of the bench: the paper's size, both end faces
    prescribed and moving apart by the pull per load step, the notch's edges
    all inside the mid-length cube layer and within the notch depth, and the
    per-material kernel supports."""
    import numpy as np

    from paper_2103_14870_amd import meshgen

    for mat, (nu, thr, radius) in meshgen.BLOCK_MATERIALS.items():
        p = meshgen.pulled_block(mat, pull=0.003, dt=0.5)
        assert p.n_tets == 168432 and p.params["damage_radius"] == radius
        assert p.params["poisson"] == nu and p.params["damage_strain"] == thr
        h, (nx, ny, nz) = p.meta["h"], p.meta["shape"]
        z = p.X[p.dir_nodes, 2]
        low = z < 0.5 * nz * h
        assert low.sum() == (~low).sum() == (nx + 1) * (ny + 1)
        # displacement per load step = velocity x dt = pull, apart
        assert np.allclose(p.dir_vel[low, 2] * p.params["dt"], -0.003)
        assert np.allclose(p.dir_vel[~low, 2] * p.params["dt"], 0.003)
        assert not p.dir_vel[:, :2].any()
        # notch: node pairs in the layer nz // 2 .. nz // 2 + 1, x below 5 cells (jitter 5 % h)
        e = p.broken_pairs
        assert e.shape[0] > 0 and (e[:, 0] < e[:, 1]).all()
        zz = p.X[e.ravel(), 2] / h
        xx = p.X[e.ravel(), 0] / h
        assert zz.min() > nz // 2 - 0.1 and zz.max() < nz // 2 + 1.1
        assert xx.max() < 5 + 0.1


def test_more_than_one_gpu_is_refused():
    """The bench times one GPU; asking for more exits with status 2 and a
    message, before any device is touched."""
    import subprocess

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""
