"""Host-side logic of bench.py that needs no GPU: the one-GPU guard, the
algorithmic byte counts and the parsing of rocprofv3 counter CSV files."""
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
    rec = {"n_dets": 1000, "spawns": 50, "merged": 40}
    b = bench.bytes_per_kernel(rec, 4096)
    assert b["k_chunk_sum"] == 4.0 * 4096
    # every slot: key 8 + accumulator 8 + population 4 + H_DD 8; population written per
    # occupied determinant, accumulator cleared and H_DD or list entry per merged target
    assert b["k_post"] == 28.0 * 4096 + 4.0 * 1000 + 16.0 * 40
    # staging key + population per slot; per spawn a key probe and an accumulator update
    assert b["k_spawn"] == 12.0 * 4096 + 24.0 * 50


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
