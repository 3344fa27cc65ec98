"""bench.py's host-side pieces (no GPU): the one-GPU guard, the traffic
figure computed from counter files, and the source digest that ties a
traffic figure to the kernel it was measured on."""
from __future__ import annotations

import json
import os
import shutil
import subprocess
import time
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

HEADER = ('"Correlation_Id","Dispatch_Id","Agent_Id","Queue_Id","Process_Id","Thread_Id","Grid_Size",'
          '"Kernel_Id","Kernel_Name","Workgroup_Size","LDS_Block_Size","Scratch_Size","VGPR_Count",'
          '"Accum_VGPR_Count","SGPR_Count","Counter_Name","Counter_Value","Start_Timestamp","End_Timestamp"\n')


def _csv(path, counter, rows):
    with open(path, "w") as f:
        f.write(HEADER)
        for i, (name, kib) in enumerate(rows):
            f.write(f'{i},{i},"Agent 1",1,1,1,256,1,"{name}",256,0,0,8,0,16,"{counter}",{kib},0,1\n')


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_from_counters(tmp_path):
    probe = "void at::native::vectorized_elementwise_kernel<4, at::native::CUDAFunctorOnSelf_add<int>>(int)"
    td = "dobfs::(anonymous namespace)::k_level_td(dobfs::GView, dobfs::WView, dobfs::KParams)"
    bu = "dobfs::(anonymous namespace)::k_level_bu(dobfs::GView, dobfs::WView, dobfs::KParams)"
    fin = "dobfs::(anonymous namespace)::k_finalize(dobfs::GView, dobfs::WView, int)"
    other = "dobfs::(anonymous namespace)::k_init_fill(dobfs::GView, dobfs::WView)"
    # a 1 MiB probe reads as 512 KiB fetched and 1024 KiB written: factors 2 and 1
    _csv(tmp_path / "f.csv", "FETCH_SIZE", [(probe, 512.0), (td, 10.0), (bu, 30.0), (other, 999.0), (td, 0.0),
                                            (bu, 20.0), (fin, 7.0)])
    _csv(tmp_path / "w.csv", "WRITE_SIZE", [(probe, 1024.0), (td, 4.0), (bu, 6.0), (td, 0.0), (bu, 10.0),
                                            (fin, 3.0)])
    out = tmp_path / "traffic.json"
    ent = bench.traffic_from_counters(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), 1 << 20, "k", str(out))
    assert ent["fetch_factor"] == pytest.approx(2.0) and ent["write_factor"] == pytest.approx(1.0)
    bu_ent = ent["kernels"]["k_level_bu"]
    assert bu_ent["launches"] == 2
    assert bu_ent["fetch_bytes_per_launch"] == round(50 * 1024 * 2 / 2)
    assert bu_ent["write_bytes_per_launch"] == round(16 * 1024 / 2)
    assert bu_ent["bytes_per_launch"] == bu_ent["fetch_bytes_per_launch"] + bu_ent["write_bytes_per_launch"]
    td_ent = ent["kernels"]["k_level_td"]
    assert td_ent["bytes_per_launch"] == round(10 * 1024 * 2 / 2) + round(4 * 1024 / 2)
    assert ent["kernels"]["k_finalize"]["launches"] == 1
    assert "k_aux" not in ent["kernels"]  # no dispatches of it in these files
    assert json.loads(out.read_text())["k"]["source_sha256"] == bench.kernel_source_digest()


def test_level_bytes_and_conversions():
    bu = {"dir": 1, "n_f": 5, "m_f": 50, "scanned": 100, "checked": 80, "found": 10}
    assert bench.bottom_up_bytes(bu, 4) == 16 * 4 + 8 * 100 + 4.125 * 80 + 8 * 10
    td = {"dir": 0, "n_f": 3, "m_f": 70_000, "scanned": 0, "checked": 30, "found": 7}
    assert bench.top_down_bytes(td) == 20 * 3 + 4.125 * 30 + 28.25 * 7
    small_td = dict(td, m_f=100)
    # level 0 never converts; after a bottom-up level, or a large top-down
    # level, the bitmap is turned into a queue; after a small top-down level
    # the queue is handed on as is
    assert bench.to_queue_bytes([td], 0, 4) == 0.0
    assert bench.to_queue_bytes([bu, td], 1, 4) == 16 * 4 + 4 * 3
    assert bench.to_queue_bytes([td, td], 1, 4) == 16 * 4 + 4 * 3
    assert bench.to_queue_bytes([small_td, td], 1, 4) == 0.0
    assert bench.to_queue_bytes([td, bu], 1, 4) == 0.0


def test_committed_traffic_matches_the_kernel_sources():
    """The HBM traffic in profiles/ was counted on the traversal kernels as
    they stand: its source digest equals the sources' (else the bench line
    would carry no traffic figure)."""
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
        tr = json.load(f)
    ent = tr["kron-s30-ef16-seed2/edge/reindex-on"]
    assert ent["source_sha256"] == bench.kernel_source_digest()
    assert ent["kernels"]["k_level_bu"]["bytes_per_launch"] > 0


def test_host_spec():
    spec = bench.host_spec()
    assert spec["nproc"] >= 1 and spec["cpus_allowed"] >= 1
    assert isinstance(spec["cpu_model"], str)


def test_source_digest_ignores_comments_only(tmp_path, monkeypatch):
    src = os.path.join(ROOT, "paper_1503_04359_amd", "csrc")
    dst = tmp_path / "paper_1503_04359_amd" / "csrc"
    dst.mkdir(parents=True)
    for f in ("bfs_kernels.hip", "device_common.h", "dobfs_internal.h"):
        shutil.copy(os.path.join(src, f), dst / f)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    base = bench.kernel_source_digest()
    p = dst / "dobfs_internal.h"
    p.write_text(p.read_text() + "\n/* a new comment */\n// and another\n")
    assert bench.kernel_source_digest() == base
    p.write_text(p.read_text() + "\nconstexpr int kUnused = 1;\n")
    assert bench.kernel_source_digest() != base


def test_harmonic_mean():
    assert bench.harmonic_mean([1.0, 1.0]) == pytest.approx(1.0)
    assert bench.harmonic_mean([1.0, 3.0]) == pytest.approx(1.5)


def test_power_sampler_mean_over_window():
    vals = iter(range(1, 10_000))
    with bench.PowerSampler(lambda: float(next(vals)), period=0.001) as ps:
        time.sleep(0.05)
        t0 = time.perf_counter()
        time.sleep(0.05)
        t1 = time.perf_counter()
        time.sleep(0.02)
    mean, n = ps.mean(t0, t1)
    inside = [w for t, w in ps.samples if t0 <= t <= t1]
    assert n == len(inside) > 0 and mean == pytest.approx(sum(inside) / len(inside))
    assert ps.mean(t1 + 10, t1 + 20) == (None, 0)


def test_hybrid_budget_leaves_top_degree_classes_on_the_host():
    import numpy as np
    import paper_1503_04359_amd as dobfs
    rng = np.random.default_rng(5)
    deg = np.concatenate([rng.integers(1, 9, 500), rng.integers(100, 5000, 20), np.zeros(30, np.int64)])
    rng.shuffle(deg)
    budget, k = bench.hybrid_budget(deg, 0.1)
    nz = int((deg > 0).sum())
    assert k == int(np.ceil(0.1 * nz))
    # brute force: order by (bit length of the degree desc, ID asc)
    order = sorted(range(deg.size), key=lambda v: (-int(deg[v]).bit_length(), v))
    host = int(sum(deg[v] for v in order[:k]))
    assert budget == dobfs.hybrid_state_bytes(deg.size) + 4 * (int(deg.sum()) - host)
    assert bench.hybrid_budget(deg, 0.0)[0] == dobfs.hybrid_state_bytes(deg.size) + 4 * int(deg.sum())
    assert bench.hybrid_budget(deg, 1.0)[0] == dobfs.hybrid_state_bytes(deg.size)
