"""Host-side pieces of the benchmark script (no GPU): the storage names reported
for skfab_info.a_format, and the lookup of recorded HBM counters, which must
give null once the kernel sources differ from the recorded hash."""
import os
import shutil

import bench


def test_storage_names():
    assert bench.storage_name(0) == "csr"
    assert bench.storage_name(1) == "sell64_int32_cols_values"
    assert bench.storage_name(2) == "sell64_int16_offsets_values"
    assert bench.storage_name(5) == "sell64_int32_cols_uint8_value_table"
    assert bench.storage_name(6) == "sell64_int16_offsets_uint8_value_table"


def test_recorded_traffic_missing_is_none():
    assert bench.recorded_traffic("no_such_workload", "fp64") is None


def test_recorded_traffic_follows_source_hash(tmp_path, monkeypatch):
    """A summary whose source hash matches the sources gives its figure; the same
    summary with another hash gives None."""
    prof = tmp_path / "profiles"
    prof.mkdir()
    for rel in bench.KERNEL_SOURCES:
        dst = tmp_path / rel
        dst.parent.mkdir(parents=True, exist_ok=True)
        shutil.copy(os.path.join(bench.ROOT, rel), dst)
    import hashlib
    h = hashlib.sha256()
    for rel in bench.KERNEL_SOURCES:
        h.update((tmp_path / rel).read_bytes())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    good = f"# header\ntraffic_bytes_per_launch: 1234\nsource_sha256: {h.hexdigest()}\n"
    (prof / "arnoldi_step_w_fp64_hbm_counters.txt").write_text(good)
    assert bench.recorded_traffic("w", "fp64") == 1234
    (prof / "arnoldi_step_w_fp64_hbm_counters.txt").write_text(good.replace(h.hexdigest(), "0" * 64))
    assert bench.recorded_traffic("w", "fp64") is None
    (prof / "arnoldi_step_b_fp64_hbm_counters.txt").write_text(
        f"traffic_bytes_per_batch: 99\nsource_sha256: {h.hexdigest()}\n")
    assert bench.recorded_traffic("b", "fp64", "traffic_bytes_per_batch") == 99
