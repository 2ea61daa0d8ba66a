"""bench.py's reading of the committed counter summaries (host only)."""
import importlib.util
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_profile_traffic_matches_source_and_tiles(tmp_path, monkeypatch):
    b = _bench()
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "eval_kernel_w_counters.md").write_text(
        "- hbm_bytes_per_launch: 2.5e+09\n- kernel_source_sha256: abc123\n"
        "- counted_tuning: K=16 P=16 C=7\n"
        "- traffic_for_tuning: K=16 P=16 C=5 bytes=1.7e+09\n")
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    assert b.profile_traffic("abc123", "w", "eval_kernel", (16, 16, 7)) == 2.5e9
    assert b.profile_traffic("abc123", "w", "eval_kernel", (16, 16, 5)) == 1.7e9
    assert b.profile_traffic("abc123", "w", "eval_kernel", (16, 16, 9)) is None   # tiles never counted
    assert b.profile_traffic("abc123", "w", "eval_kernel") == 2.5e9               # no tiles asked for
    assert b.profile_traffic("ffff00", "w", "eval_kernel", (16, 16, 7)) is None   # another kernel source
    assert b.profile_traffic("abc123", "missing", "eval_kernel") is None


def test_committed_summaries_parse():
    b = _bench()
    for kernel in ("eval_kernel", "batch_pass", "points_eval_kernel", "small_run_kernel"):
        assert len(b.kernel_source_sha(kernel)) == 16
