"""bench.py takes per-launch counter figures (HBM bytes, executed MFMA flops)
from the committed rocprofv3 summaries only while the kernel sources are the
ones those counters were taken on; otherwise it reports them as null."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _summary(path, key, value, sha):
    with open(path, "w") as f:
        f.write(f"# summary\n\nsome text: with a colon\n{key}: {value}\n"
                f"kernel_sources_sha256: `{sha}`\n")


def test_field_read_when_sources_match(tmp_path):
    p = str(tmp_path / "s.md")
    _summary(p, "traffic_bytes_per_launch", "3.5e+11", bench.kernel_sources_sha256())
    assert bench._profile_field(p, "traffic_bytes_per_launch") == pytest.approx(3.5e11)


def test_field_null_when_sources_changed(tmp_path):
    p = str(tmp_path / "s.md")
    _summary(p, "traffic_bytes_per_launch", "3.5e+11", "0" * 64)
    assert bench._profile_field(p, "traffic_bytes_per_launch") is None


def test_field_null_when_missing(tmp_path):
    p = str(tmp_path / "s.md")
    _summary(p, "other_field", "1.0", bench.kernel_sources_sha256())
    assert bench._profile_field(p, "traffic_bytes_per_launch") is None
    assert bench._profile_field(str(tmp_path / "absent.md"), "x") is None


@pytest.mark.parametrize("path,key", [
    (bench.TRAFFIC_FILE, "traffic_bytes_per_launch"),
    (bench.MFMA_FILE, "mfma_flops_per_launch"),
])
def test_committed_summaries_carry_their_fields(path, key):
    # the committed summaries name the figure the bench reads and the hash of
    # the kernel sources they were measured on
    with open(path) as f:
        text = f.read()
    keys = {line.split(":", 1)[0].strip() for line in text.splitlines() if ":" in line}
    assert key in keys and "kernel_sources_sha256" in keys
