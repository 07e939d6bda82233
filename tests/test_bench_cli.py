"""bench.py's command line on the CPU: more than one GPU is refused before
anything touches a device (the library has no multi-GPU path)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args, env=None):
    e = dict(os.environ)
    e.update(env or {})
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, env=e)


def test_more_than_one_gpu_is_refused():
    r = _bench("--gpus", "2")
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout == ""  # no JSON line


def test_world_size_above_one_is_refused():
    r = _bench(env={"WORLD_SIZE": "4"})
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr


def test_help_lists_the_contract_flags():
    r = _bench("--help")
    assert r.returncode == 0
    for flag in ("--gpus", "--steps", "--warmup", "--workload"):
        assert flag in r.stdout


def test_traffic_is_null_once_the_kernel_sources_change(tmp_path, monkeypatch):
    # a counter summary carries a hash of the sources its kernel is built
    # from; once one of them changes, bench.py reports traffic as null, and
    # a change to another kernel's source leaves it valid
    import hashlib
    import shutil
    sys.path.insert(0, ROOT)
    import bench
    csrc = tmp_path / "paper_2301_09125_amd" / "csrc"
    shutil.copytree(os.path.join(ROOT, "paper_2301_09125_amd", "csrc"), csrc)
    h = hashlib.sha256()
    for f in sorted(["lpa_vote.hip", "lpa_vote_dev.h", "lpa_device.h", "lpa_internal.h"]):
        h.update((csrc / f).read_bytes())
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "traffic_vote_hub_toy.txt").write_text(
        "# toy summary\nkernel: vote_hub\ntraffic_bytes_per_launch: 12345\n"
        f"kernel_sources_sha256: {h.hexdigest()[:16]}\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.traffic_from_profile("toy", "vote_hub") == 12345
    assert bench.traffic_from_profile("other", "vote_hub") is None  # no summary
    with open(csrc / "lpa_copra.hip", "a") as f:
        f.write("\n// changed\n")
    assert bench.traffic_from_profile("toy", "vote_hub") == 12345
    with open(csrc / "lpa_vote.hip", "a") as f:
        f.write("\n// changed\n")
    assert bench.traffic_from_profile("toy", "vote_hub") is None


@pytest.mark.gpu
def test_bench_gather_probe():
    """The bench-only random-gather probe (bench_gather_probe.hip, not part of
    liblpa.so): a positive rate, indices past the table clamped into it, and
    an empty index stream rejected."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import bench
    probe = bench.GatherProbe()
    idx = torch.randint(0, 1 << 20, (1 << 20,), dtype=torch.int32, device="cuda")
    table = torch.zeros(1 << 16, dtype=torch.int32, device="cuda")  # most indices past the end: clamped
    assert probe.rate(idx, table, reps=2) > 0
    with pytest.raises(RuntimeError):
        probe.rate(idx[:0], table)
