"""Host-side logic of the benchmark (CPU): the one-GPU guard and the rule that HBM traffic is reported
only from a profile of the same workload, kernel sources, instance and tuning."""
import hashlib
import json
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _record(tmp_path, sha, instance, tuning, workload="box"):
    d = tmp_path / "profiles"
    d.mkdir()
    rec = {"kernel": "gather_update_kernel", "workload": workload, "instance": instance, "tuning": tuning,
           "source_sha256_16": sha, "avg_launch_ms": 1.0, "traffic_bytes_per_launch": 123456}
    (d / "gather_traffic.md").write_text("# profile\n\n```\n" + json.dumps(rec) + "\n```\n")


def _sources_sha():
    h = hashlib.sha256()
    for f in ["hk_gather.hip", "hk_internal.h", "hk_kernels.h", "hk_fquant.h"]:
        h.update(open(os.path.join(ROOT, "paper_2504_04411_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


@pytest.fixture
def bench_mod():
    sys.path.insert(0, ROOT)
    import bench
    return bench


def test_traffic_only_for_the_profiled_sources_instance_and_tuning(tmp_path, bench_mod, monkeypatch):
    tun = {"cell_scale": 0.699999988079071, "heavy_cost": 2048, "lanes_light": 16, "lanes_heavy": 64}
    inst = "gather_update_kernel<true,false,1,16,64>"
    _record(tmp_path, _sources_sha(), inst, [0.7, 2048, 16, 64])
    # the record is read relative to the repository root; point it at the temporary copy
    for f in ["hk_gather.hip", "hk_internal.h", "hk_kernels.h", "hk_fquant.h"]:
        os.makedirs(tmp_path / "paper_2504_04411_amd" / "csrc", exist_ok=True)
        (tmp_path / "paper_2504_04411_amd" / "csrc" / f).write_bytes(
            open(os.path.join(ROOT, "paper_2504_04411_amd", "csrc", f), "rb").read())
    monkeypatch.setattr(bench_mod, "ROOT", str(tmp_path))
    assert bench_mod.profiled_traffic("box", inst, tun) == 123456
    assert bench_mod.profiled_traffic("sets", inst, tun) is None
    assert bench_mod.profiled_traffic("box", "gather_update_kernel<true,false,1,8,64>", tun) is None
    assert bench_mod.profiled_traffic("box", inst, dict(tun, heavy_cost=4096)) is None
    # a changed source invalidates the record
    p = tmp_path / "paper_2504_04411_amd" / "csrc" / "hk_gather.hip"
    p.write_bytes(p.read_bytes() + b"\n")
    assert bench_mod.profiled_traffic("box", inst, tun) is None
