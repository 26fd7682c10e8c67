"""The autotuner's table is tied to the device sources it was measured on
(no GPU needed for these checks)."""
import json

from paper_1702_03484_amd import autotune
from paper_1702_03484_amd.profile_summary import kernel_sha


def test_install_refuses_a_table_from_other_kernel_sources(tmp_path):
    stale = tmp_path / "stale.json"
    stale.write_text(json.dumps({"kernel_source_sha256": "0" * 64,
                                 "sort": {"20:11": {"radix_bits": 5, "keys_per_thread": 8}}}))
    # refused before the session is touched
    assert autotune.install(None, str(stale)) is False
    legacy = tmp_path / "legacy.json"  # a table without a source hash
    legacy.write_text(json.dumps({"20:11": {"radix_bits": 5, "keys_per_thread": 8}}))
    assert autotune.install(None, str(legacy)) is False
    assert autotune.install(None, str(tmp_path / "missing.json")) is False


def test_install_accepts_a_table_of_these_sources(tmp_path):
    fresh = tmp_path / "fresh.json"
    fresh.write_text(json.dumps({"kernel_source_sha256": kernel_sha(), "sort": {}, "materialize": {}}))
    assert autotune.install(None, str(fresh)) is True
