"""Host-side logic of bench.py that needs no GPU: the one-GPU guard, the
algorithmic byte counts, the averaging start and the parsing of rocprofv3
counter CSV files."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]


def test_algorithmic_bytes():
    # two iterations: the main list read before each is the previous iteration's
    recs = [{"n_dets": 1100, "spawns": 50, "merged": 40, "born": 30},
            {"n_dets": 1200, "spawns": 60, "merged": 45, "born": 35}]
    group, post = bench.method_bytes(recs, 1000)
    # per occupied determinant 21 B read + 4 B written; per spawn record 16 B read;
    # per merged target 16 B; per new determinant 20 B
    p1 = 25.0 * 1000 + 16.0 * 50 + 16.0 * 40 + 20.0 * 30
    p2 = 25.0 * 1100 + 16.0 * 60 + 16.0 * 45 + 20.0 * 35
    assert post == (p1 + p2) / 2
    # the partition by bucket adds 32 B per spawn record (read + write)
    assert group == (p1 + 32.0 * 50 + p2 + 32.0 * 60) / 2


def test_avg_start_is_one_unit_of_imaginary_time():
    class P:
        tau = 5e-4
    assert bench.avg_start_for(P) == 2000
    P.tau = 0.01
    assert bench.avg_start_for(P) == 200


def test_counter_csv_means(tmp_path):
    rows = ["Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value"]
    # k_post: dispatches 1..4 with FETCH_SIZE 10, 20, 30, 40 (one dispatch split over two rows)
    for disp, v in ((1, 10.0), (2, 20.0), (3, 30.0), (4, 40.0)):
        rows.append(f'{disp},"fq::k_post(fq::EngineArgs, fq::SysDesc const*)",FETCH_SIZE,{v / 2}')
        rows.append(f'{disp},"fq::k_post(fq::EngineArgs, fq::SysDesc const*)",FETCH_SIZE,{v / 2}')
    rows.append('5,"fq::k_spawn(fq::EngineArgs, fq::SysDesc const*)",FETCH_SIZE,7')
    sub = tmp_path / "run" / "host"
    sub.mkdir(parents=True)
    (sub / "f_counter_collection.csv").write_text("\n".join(rows) + "\n")
    allm = bench.pmc_means(str(tmp_path))
    assert allm[("fq::k_post", "FETCH_SIZE")] == (25.0, 4)
    assert allm[("fq::k_spawn", "FETCH_SIZE")] == (7.0, 1)
    last2 = bench.pmc_means(str(tmp_path), 2)
    assert last2[("fq::k_post", "FETCH_SIZE")] == (35.0, 2)
