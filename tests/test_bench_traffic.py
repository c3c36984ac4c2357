"""Host-side checks of how bench.py reports HBM traffic (no GPU needed).

The bench line carries the counter-measured bytes of the dominant kernel
only while the committed record was taken on the current kernel sources and
for the schedule the run used; in every other case it must report null
rather than a stale figure.
"""

import importlib.util
import json
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _tree(tmp_path, kernels=b"kernel v1", plan=b"plan v1"):
    csrc = tmp_path / "paper_1703_03637_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "kernels.hip").write_bytes(kernels)
    (csrc / "plan.cpp").write_bytes(plan)
    (tmp_path / "profiles").mkdir()
    return tmp_path


SCHED = {"windowed": 1, "window_kb": 1024, "max_passes": 2, "lanes_per_row": 4, "blocks_per_cu": 0,
         "stage_tables": 1, "nt_streams": 1, "sector_blocks": 0, "us": 4900}


def _record(b, tmp_path, hash_value, key="1,1024,2,4,0,1,1", nbytes=30.8e9):
    rec = {"kernel_source_hash": hash_value, "schedules": {key: {"hbm_bytes_per_product": nbytes}}}
    (tmp_path / "profiles" / "traffic_kh_honeycomb24_tpq_b16_c64.json").write_text(json.dumps(rec))


def test_traffic_reported_for_matching_sources_and_schedule(tmp_path, monkeypatch):
    b = _bench()
    monkeypatch.setattr(b, "ROOT", str(_tree(tmp_path)))
    _record(b, tmp_path, b.kernel_source_hash())
    assert b.measured_traffic(SCHED) == 30.8e9


def test_traffic_null_after_a_kernel_source_change(tmp_path, monkeypatch):
    b = _bench()
    monkeypatch.setattr(b, "ROOT", str(_tree(tmp_path)))
    _record(b, tmp_path, b.kernel_source_hash())
    (tmp_path / "paper_1703_03637_amd" / "csrc" / "plan.cpp").write_bytes(b"plan v2")
    assert b.measured_traffic(SCHED) is None


def test_traffic_null_for_another_schedule_or_no_record(tmp_path, monkeypatch):
    b = _bench()
    monkeypatch.setattr(b, "ROOT", str(_tree(tmp_path)))
    assert b.measured_traffic(SCHED) is None                      # no record at all
    _record(b, tmp_path, b.kernel_source_hash(), key="1,2048,2,4,0,1,1")
    assert b.measured_traffic(SCHED) is None
    (tmp_path / "profiles" / "traffic_kh_honeycomb24_tpq_b16_c64.json").write_text("{not json")
    assert b.measured_traffic(SCHED) is None


def test_schedule_keys_of_pinned_and_tuned_schedules():
    b = _bench()
    assert b.schedule_key(SCHED) == "1,1024,2,4,0,1,1"
    # a pinned schedule of 5 or 6 fields takes the defaults of the fields it omits
    assert b.schedule_key({"pinned": "1,1024,2,4,0"}) == "1,1024,2,4,0,1,1"
    assert b.schedule_key({"pinned": "1,1024,2,4,0,1"}) == "1,1024,2,4,0,1,1"
    assert b.schedule_key({"pinned": "1,1024,2,4,0,1,0"}) == "1,1024,2,4,0,1,0"


def test_committed_record_names_a_measured_schedule():
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic_kh_honeycomb24_tpq_b16_c64.json")))
    assert len(rec["kernel_source_hash"]) == 16
    assert "1,1024,2,4,0,1,1" in rec["schedules"]
    for e in rec["schedules"].values():
        assert e["hbm_bytes_per_product"] == e["fetch_bytes_per_product"] + e["write_bytes_per_product"]
        assert e["hbm_bytes_per_product"] > 4.29e9   # at least the compulsory bytes of one product
