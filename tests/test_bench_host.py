"""Host logic of the measurement: the one-GPU guard of bench.py, its
algorithmic byte counts (the per-row formulas of the kernels, checked at the
sizes the profiles report), and the rocprofv3 summaries' kernel naming and
counter calibration."""
import csv
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1608_01906_amd import profiling  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout == ""


# channel: D2Q9, ELL width 7, five basis matrices, FP32 values and populations
CH = dict(Q=9, D=2, W=7, NB=5, s=4, sp=4, dev=True)
# 3-D droplet: D3Q19, width 15, nine basis matrices
D3 = dict(Q=19, D=3, W=15, NB=9, s=4, sp=4, dev=True)


@pytest.mark.parametrize("cls,per_row", [
    # 16 moving populations of 4 bytes; pattern 6 off-diagonal x 4 B; mass values 7 x 4 B; 1/m 4 B
    ("cg_b", 3 * 64 + 24 + 28 + 4),          # read p r, write r (x formed by cg_x)
    ("cg_a", 3 * 64 + 24 + 28 + 4),          # read r p_old, write p_new
    ("cg_init", 2 * 64 + 24 + 28 + 4),       # read rhs, write r
    ("cheb", 4 * 64 + 24 + 28 + 4),          # read x_k rhs x_{k-1}, write x_{k+1}
    ("lumped", 2 * 64 + 4),
    # 16 stored deviations + 2 references, pattern, 5 x 6 off-diagonal basis values, 16 rhs values
    ("stream", 64 + 8 + 24 + 5 * 6 * 4 + 64),
])
def test_channel_bytes_per_row(cls, per_row):
    assert bench.kernel_bytes(cls, **CH) == per_row


def test_bytes_per_launch_match_the_reported_figures():
    """The per-launch figures quoted with the profiles: fused cg_b on the
    262,144-row channel, and the 3-D cg_a averaged over 17 iterations (the
    first one reads no previous direction)."""
    assert bench.kernel_bytes("cg_b", **CH) * 262144 == 65011712
    # x = rhs / m + sum of the 15 stored directions: read rhs, 1/m and 15 directions, write x
    assert bench.kernel_bytes("cg_x", K=15, **CH) == 17 * 64 + 4
    # 3-D (recurrence form): cg_a reads r p q and writes p q, the first of
    # 17 iterations reads r only; cg_b streams q r, writes r
    first = 1.0 / 17
    per_launch = bench.kernel_bytes("cg_a", first_frac=first, **D3) * 2097152
    assert abs(per_launch - ((5 - 2 / 17) * 144 + 56 + 60 + 4) * 2097152) < 1.0
    assert bench.kernel_bytes("cg_b", **D3) == 3 * 144 + 4
    # first iteration of cg_a in 2-D: two population passes instead of three
    assert bench.kernel_bytes("cg_a", first_frac=1.0, **CH) == 2 * 64 + 56


def test_fp64_plain_bytes():
    """FP64 plain: 8-byte values and populations, no references."""
    f64 = dict(Q=9, D=2, W=7, NB=5, s=8, sp=8, dev=False)
    assert bench.kernel_bytes("cg_b", **f64) == 3 * 128 + 24 + 56 + 8
    # plain populations: the diagonal coefficients are read
    assert bench.kernel_bytes("stream", **f64) == 128 + 24 + 5 * 7 * 8 + 128


@pytest.mark.parametrize("name,cls", [
    ("void fel::k_cg_a_fused<float, 7, 16, 1>(fel::DevLayout, int)", "cg_a"),
    ("void fel::k_cg_b_lds<double, 15, 36, 2>(fel::DevLayout, int, int)", "cg_b"),
    ("void fel::k_cg_init<float, 7, 16, 2>(fel::DevLayout, int)", "cg_init"),
    ("void fel::k_cheb_first_lds<float, 7, 16, 4>(fel::DevLayout, int, int, double)", "cheb"),
    ("void fel::k_cheb<float, 7, 16, 2>(fel::DevLayout, int, int, double, double)", "cheb"),
    ("void fel::k_cg_x<float, 16>(fel::DevLayout, int, int)", "cg_x"),
    ("void fel::k_finalize<36>(fel::DevLayout, int, int)", "finalize"),
    ("void fel::k_stream_dev<9, 7, float>(fel::DevLayout, int)", "stream"),
    ("void fel::k_collide_plain<19, 15>(fel::DevLayout, int)", "collide"),
    ("void fel::k_moments_dev<9, float>(fel::DevLayout, int)", "moments"),
    ("__amd_rocclr_copyBuffer", None),
])
def test_kernel_class(name, cls):
    assert profiling.kernel_class(name) == cls


def test_solver_kernel_name():
    assert profiling.solver_kernel_name("cg_b", "fp32", 7, 16, 1, False, True) == "fel::k_cg_b_fused<float, 7, 16, 1>"
    # staged kernels: 2 halo rounds when the largest halo fits in 2 tiles of 256 rows, else 4
    assert profiling.solver_kernel_name("cg_a", "fp64", 15, 36, 2, True, halo_max=1024) == \
        "fel::k_cg_a_lds<double, 15, 36, 2, 4>"
    assert profiling.solver_kernel_name("cg_a", "fp32", 7, 16, 2, True, halo_max=266) == \
        "fel::k_cg_a_lds<float, 7, 16, 2, 2>"
    assert profiling.solver_kernel_name("cg_b", "fp32", 7, 16, 4, True, halo_max=512) == \
        "fel::k_cg_b_lds<float, 7, 16, 4, 2>"
    assert profiling.solver_kernel_name("cg_b", "fp32", 7, 16, 4, True, halo_max=516) == \
        "fel::k_cg_b_lds<float, 7, 16, 4, 4>"
    # the per-wavefront stage: halo rounds 0 whatever the tile halos
    assert profiling.solver_kernel_name("cg_a", "fp32", 7, 16, 2, "wave", halo_max=266) == \
        "fel::k_cg_a_lds<float, 7, 16, 2, 0>"
    assert profiling.solver_kernel_name("cg_a", "fp32", 7, 16, 4, False) == "fel::k_cg_a<float, 7, 16, 4>"
    # the Chebyshev kernels have no fused form
    assert profiling.solver_kernel_name("cheb", "fp32", 7, 16, 2, False, True) == "fel::k_cheb<float, 7, 16, 2>"


def _counter_csv(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, v in rows:
            w.writerow(dict(Kernel_Name=name, Counter_Name=counter, Counter_Value=v))


def test_traffic_calibration(tmp_path):
    """A 256 MiB device copy that reads FETCH_SIZE = half its bytes and
    WRITE_SIZE exactly gives factors 2 and 1; a kernel's traffic is then
    fetch x 2 + write x 1, per instantiation, averaged over its dispatches."""
    name = "void fel::k_cg_b_fused<float, 7, 16, 1>(fel::DevLayout, int)"
    other = "void fel::k_cg_b<float, 7, 16, 2>(fel::DevLayout, int, int)"
    fetch, write = tmp_path / "f.csv", tmp_path / "w.csv"
    _counter_csv(fetch, "FETCH_SIZE", [(profiling.COPY_KERNEL, 131072.0), (name, 1000.0), (name, 1200.0),
                                       (other, 10.0)])
    _counter_csv(write, "WRITE_SIZE", [(profiling.COPY_KERNEL, 262144.0), (name, 500.0), (name, 500.0),
                                       (other, 20.0)])
    rec = profiling.traffic(str(fetch), str(write), 256, "channel2d", "fp32", 0, ["cmd"])
    assert rec["fetch_factor"] == 2.0 and rec["write_factor"] == 1.0
    assert rec["kernel_source_sha256_16"] == profiling.device_source_hash()
    k = rec["kernels"]["cg_b"]["fel::k_cg_b_fused<float, 7, 16, 1>"]
    assert k["dispatches"] == 2
    assert k["traffic_bytes"] == (1100 * 2 + 500) * 1024
    assert profiling.lookup_traffic(rec, "cg_b", "fel::k_cg_b_fused<float, 7, 16, 1>") == k["traffic_bytes"]
    assert profiling.lookup_traffic(rec, "cg_b", "fel::k_cg_b<float, 7, 16, 2>") == (10 * 2 + 20) * 1024
    # the most dispatched instantiation when no name is given
    assert profiling.lookup_traffic(rec, "cg_b") == k["traffic_bytes"]
    assert profiling.lookup_traffic(rec, "cg_a") is None


def test_traffic_needs_the_copy_probe(tmp_path):
    fetch, write = tmp_path / "f.csv", tmp_path / "w.csv"
    name = "void fel::k_cg_b<float, 7, 16, 2>(fel::DevLayout, int, int)"
    _counter_csv(fetch, "FETCH_SIZE", [(name, 10.0)])
    _counter_csv(write, "WRITE_SIZE", [(name, 20.0)])
    with pytest.raises(SystemExit):
        profiling.traffic(str(fetch), str(write), 256, "channel2d", "fp32", 0, [])


def test_measured_traffic_only_for_current_sources(tmp_path, monkeypatch):
    """bench.py takes measured traffic from a committed summary only while
    the device sources hash as when the counters were taken (else null)."""
    import json
    (tmp_path / "profiles").mkdir()
    rec = dict(kernel_source_sha256_16=profiling.device_source_hash(),
               kernels={"cg_b": {"fel::k_cg_b<float, 7, 16, 2>": dict(dispatches=4, traffic_bytes=123)}})
    path = tmp_path / "profiles" / "channel2d_traffic_fp32_mass0.json"
    path.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("channel2d", "fp32", 0, "cg_b", "fel::k_cg_b<float, 7, 16, 2>") == 123
    assert bench.measured_traffic("channel2d", "fp32", 0, "cg_b", "fel::k_cg_b<float, 7, 16, 4>") is None
    assert bench.measured_traffic("channel2d", "fp32", 2, "cg_b", None) is None  # no summary
    # a summary serves only the device row order it was taken on
    assert bench.measured_traffic("channel2d", "fp32", 0, "cg_b", "fel::k_cg_b<float, 7, 16, 2>", 1) is None
    zpath = tmp_path / "profiles" / "channel2d_traffic_fp32_mass0_zorder.json"
    zpath.write_text(json.dumps(dict(rec, node_order=1)))
    assert bench.measured_traffic("channel2d", "fp32", 0, "cg_b", "fel::k_cg_b<float, 7, 16, 2>", 1) == 123
    zpath.write_text(json.dumps(dict(rec, node_order=0)))
    assert bench.measured_traffic("channel2d", "fp32", 0, "cg_b", "fel::k_cg_b<float, 7, 16, 2>", 1) is None
    rec["kernel_source_sha256_16"] = "0" * 16
    path.write_text(json.dumps(rec))
    assert bench.measured_traffic("channel2d", "fp32", 0, "cg_b", "fel::k_cg_b<float, 7, 16, 2>") is None


@pytest.mark.parametrize("D,precision,k,mass_mode,expect", [
    (2, "fp64", 30, 0, 31020), (2, "fp32", 15, 0, 8688), (2, "fp32_fp16", 15, 0, 8562),
    (3, "fp64", 34, 0, 74144), (3, "fp32", 17, 0, 20712),
    (2, "fp32", 15, 1, 960), (3, "fp32", 17, 1, 2368)])
def test_whole_step_byte_model(D, precision, k, mass_mode, expect):
    """The whole-step bytes per node of the measurement's byte model, at the
    figures it tabulates (FP64 plain, FP32, FP16 storage; lumped mass)."""
    assert bench.survey_bytes_per_node(D, precision, k, mass_mode) == expect


def test_whole_step_byte_model_has_no_chebyshev_figure():
    assert bench.survey_bytes_per_node(2, "fp32", 15, 2) is None
