"""Host-side checks of the measurement records bench.py reads (no GPU): every
HBM-traffic record named in bench.TRAFFIC exists under profiles/, parses, and
lists the same kernel sources that bench.py hashes.  A record whose sources
have changed since it was measured is reported (bench.py then prints a null
traffic) rather than failed: only a GPU run can re-measure it."""
import os
import re
import sys
import warnings

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def parse(path):
    rec = {}
    with open(path) as fh:
        for line in fh:
            m = re.match(r"^- (\w+): (.*)$", line.strip())
            if m:
                rec[m.group(1)] = m.group(2)
    return rec


def test_traffic_records_exist_and_name_their_sources():
    assert bench.TRAFFIC, "no traffic records declared"
    for kernel, (fname, sources) in bench.TRAFFIC.items():
        path = os.path.join(ROOT, "profiles", fname)
        assert os.path.exists(path), (kernel, path)
        rec = parse(path)
        assert re.fullmatch(r"`?[0-9a-f]{64}`?", rec.get("source_sha256", "")), (kernel, rec)
        assert float(rec["traffic_bytes_per_launch"].strip("`")) > 0, (kernel, rec)
        listed = re.findall(r"`([^`]+)`", rec.get("sources", ""))
        assert sorted(listed) == sorted(sources), (kernel, listed, sources)
        for src in sources:
            assert os.path.exists(os.path.join(ROOT, src)), (kernel, src)
        # the command that produced the record is part of the record
        with open(path) as fh:
            text = fh.read()
        assert "rocprofv3 --pmc FETCH_SIZE" in text and "rocprofv3 --pmc WRITE_SIZE" in text, kernel


def test_traffic_records_match_current_sources_or_warn():
    for kernel in bench.TRAFFIC:
        if bench.recorded_traffic(4096, kernel) is None:
            warnings.warn(f"traffic record of {kernel} predates its current sources; "
                          "bench.py reports null traffic for it until it is re-measured")
    # a record is only ever used at the size it was measured at
    assert all(bench.recorded_traffic(1024, k) is None for k in bench.TRAFFIC)
