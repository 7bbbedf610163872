"""The bench's counter records (CPU only): a traffic record is used only when
it was taken on the current kernel sources and the same launch shape; the
reverse step's records hash its own kernel as well; every committed record
names a command that runs committed files."""
import glob
import importlib.util
import json
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
_spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
bench = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(bench)

LAUNCH = {"threads": 768, "tile_bytes": 29584, "units": 1000}


def _write(path, source_hash, launch, nbytes):
    with open(path, "w") as fh:
        json.dump({"source_hash": source_hash, "launch": launch, "bytes_per_launch": nbytes}, fh)


def test_traffic_record_used_only_when_current(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_FILE",
                        str(tmp_path / "traffic_{kernel}_{workload}_{dtype}.json"))
    path = tmp_path / "traffic_k_step_fused_w_f64.json"
    # no record
    assert bench.load_traffic("w", "f64", LAUNCH) == (None, None)
    # current sources, same launch shape
    _write(path, bench.kernel_source_hash(), LAUNCH, 123.0)
    got, src = bench.load_traffic("w", "f64", LAUNCH)
    assert got == 123.0 and src.endswith("traffic_k_step_fused_w_f64.json")
    # another launch shape
    other = dict(LAUNCH, units=999)
    got, note = bench.load_traffic("w", "f64", other)
    assert got is None and "launch shape" in note
    # sources changed since
    _write(path, "0" * 16, LAUNCH, 123.0)
    got, note = bench.load_traffic("w", "f64", LAUNCH)
    assert got is None and note.startswith("stale")


def test_reverse_records_hash_the_reverse_kernel(tmp_path, monkeypatch):
    assert "paper_1612_03399_amd/csrc/k_backward.hip" in bench.REVERSE_SOURCES
    assert set(bench.KERNEL_SOURCES) <= set(bench.REVERSE_SOURCES)
    h_step = bench.kernel_source_hash()
    h_rev = bench.kernel_source_hash(bench.REVERSE_SOURCES)
    assert h_step != h_rev
    monkeypatch.setattr(bench, "TRAFFIC_FILE",
                        str(tmp_path / "traffic_{kernel}_{workload}_{dtype}.json"))
    path = tmp_path / "traffic_k_step_vjp_fused_w_f64.json"
    # a record taken on the step's hash alone does not pass for the reverse step
    _write(path, h_step, LAUNCH, 7.0)
    got, note = bench.load_traffic("w", "f64", LAUNCH, kernel="k_step_vjp_fused",
                                   sources=bench.REVERSE_SOURCES)
    assert got is None and note.startswith("stale")
    _write(path, h_rev, LAUNCH, 7.0)
    got, _ = bench.load_traffic("w", "f64", LAUNCH, kernel="k_step_vjp_fused",
                                sources=bench.REVERSE_SOURCES)
    assert got == 7.0


def test_committed_records_name_committed_commands():
    paths = sorted(glob.glob(os.path.join(ROOT, "profiles", "traffic_*.json")) +
                   glob.glob(os.path.join(ROOT, "profiles", "valu_*.json")))
    assert paths
    for p in paths:
        with open(p) as fh:
            rec = json.load(fh)
        cmds = rec.get("commands") or [rec.get("command")]
        assert cmds and all(cmds), p
        for c in cmds:
            assert c.startswith("rocprofv3 --pmc "), (p, c)
            prog = c.split(" -- ", 1)[1].split()
            assert prog[0] == "python3" and os.path.exists(os.path.join(ROOT, prog[1])), (p, c)
            assert "_work" not in c, (p, c)
        assert len(rec["source_hash"]) == 16, p
        assert {"threads", "tile_bytes", "units"} <= set(rec["launch"]), p
