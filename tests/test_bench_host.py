"""Host logic of the benchmark: the HBM traffic figure is taken from a committed counter summary
only for the kernel sources and the tuner variant the counters were taken on."""
import os

import bench


def _tree(tmp_path, monkeypatch, text):
    (tmp_path / "profiles").mkdir()
    pkg = tmp_path / "paper_1912_07645_amd"
    pkg.mkdir()
    os.symlink(os.path.join(bench.ROOT, "paper_1912_07645_amd", "csrc"), pkg / "csrc")
    (tmp_path / "profiles" / "s.md").write_text(text)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setitem(bench.PROFILE_SUMMARY, "kh2d", "s.md")


def test_traffic_is_keyed_by_variant(tmp_path, monkeypatch):
    h = bench.kernel_sources_hash("kh2d")
    _tree(tmp_path, monkeypatch,
          f"sources_sha256: {h}\ntraffic_variant: 0\ntraffic_bytes_per_launch: 100\n\n"
          "traffic_bytes_per_launch[variant 3]: 300\n")
    assert bench.measured_traffic("kh2d", 0) == 100.0
    assert bench.measured_traffic("kh2d", 3) == 300.0
    assert bench.measured_traffic("kh2d", 1) is None


def test_traffic_needs_the_current_sources_and_a_named_variant(tmp_path, monkeypatch):
    _tree(tmp_path, monkeypatch,
          "sources_sha256: 0123456789abcdef\ntraffic_variant: 0\ntraffic_bytes_per_launch: 100\n")
    assert bench.measured_traffic("kh2d", 0) is None        # counters of other sources
    h = bench.kernel_sources_hash("kh2d")
    (tmp_path / "profiles" / "s.md").write_text(f"sources_sha256: {h}\ntraffic_bytes_per_launch: 100\n")
    assert bench.measured_traffic("kh2d", 0) is None        # variant not named


def test_committed_headline_summary_covers_both_variants():
    h = bench.kernel_sources_hash("kh2d")
    text = open(os.path.join(bench.ROOT, "profiles", bench.PROFILE_SUMMARY["kh2d"])).read()
    if f"sources_sha256: {h}" in text:
        assert bench.measured_traffic("kh2d", 0) is not None
        assert bench.measured_traffic("kh2d", 1) is not None


def test_stats_traffic_follows_the_statistics_sources(tmp_path, monkeypatch):
    h = bench.sources_hash(bench.STATS_KERNEL_SOURCES)
    _tree(tmp_path, monkeypatch, "")
    (tmp_path / "profiles" / bench.STATS_SUMMARY).write_text(
        f"sources_sha256: {h}\ntraffic_bytes_per_call: 123\n")
    assert bench.measured_stats_traffic() == 123.0
    (tmp_path / "profiles" / bench.STATS_SUMMARY).write_text(
        "sources_sha256: 0123456789abcdef\ntraffic_bytes_per_call: 123\n")
    assert bench.measured_stats_traffic() is None
