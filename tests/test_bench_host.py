"""Host-side pieces of the benchmark script: the committed counter summaries
it reads its traffic figure from."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_clip_traffic_summary_is_found_and_complete():
    # the default workload's summary must resolve to a committed file that
    # carries both the source hash and the figure; whether the hash still
    # matches the clip sources is up to the last counter run
    wl = "cluster-16m-f32"
    path = bench.clip_traffic_profile(wl)
    assert os.path.isfile(path), path
    vals = bench.clip_traffic_fields(wl)
    assert len(vals.get("clip sources sha256", "")) == 64
    assert float(vals["bytes per step"]) > 0
    if vals["clip sources sha256"] == bench.clip_sources_sha256():
        assert bench.clip_traffic(wl) == float(vals["bytes per step"])
    else:
        assert bench.clip_traffic(wl) is None


def test_more_than_one_gpu_is_refused(capsys):
    # the tessellation runs on one GPU; asking for more ends with a message
    # before anything touches the device
    assert bench.main(["--gpus", "2"]) == 2
    assert "one GPU only" in capsys.readouterr().err
