"""CPU checks of the benchmark's bookkeeping: the key under which stored
counter traffic is matched to the dominant kernel's sources, and the
records committed under profiles/."""

import glob
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_code_tokens_ignore_comments_and_layout_only():
    a = "int f(int x) {\n    // scale\n    return 2 * x; /* twice */\n}\n"
    b = "int f(int x) {   return 2 * x;\n}  // another comment\n"
    c = "int f(int x) {\n    return 3 * x;\n}\n"
    assert bench.code_tokens(a) == bench.code_tokens(b)
    assert bench.code_tokens(a) != bench.code_tokens(c)
    # a block comment spanning lines and a line comment with code after it
    assert bench.code_tokens("a /* x\n y */ b") == "a b"
    assert bench.code_tokens("a // x\nb") == "a b"


def test_traffic_records_are_consistent_with_the_kernel_code():
    recs = sorted(glob.glob(os.path.join(ROOT, "profiles", "traffic_*.json")))
    assert recs, "no traffic records under profiles/"
    stale = []
    for path in recs:
        rec = json.load(open(path))
        dim = 3 if rec["kernel"].startswith("k3_") else 2
        # the scaled counter bytes add up, and the copy calibration is the one stated
        assert abs(rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"] -
                   rec["bytes_per_launch"]) < 1e-6 * rec["bytes_per_launch"]
        cr = rec["copy_reference"]
        assert abs(cr["fetch_scale"] * cr["fetch_kib"] * 1024 - cr["bytes_read"]) < 1e-6 * cr["bytes_read"]
        assert abs(cr["write_scale"] * cr["write_kib"] * 1024 - cr["bytes_written"]) < 1e-6 * cr["bytes_written"]
        wl, prec = rec["workload"], rec["precision"]
        if rec["kernel_source_hash"] == bench.kernel_source_hash(dim):
            assert bench.stored_traffic(dim, wl, prec) == rec["bytes_per_launch"]
        else:
            # counters taken before the kernel's code changed: reported as null
            assert bench.stored_traffic(dim, wl, prec) is None
            stale.append(os.path.basename(path))
    if stale:
        pytest.skip("counter records older than the kernel code (traffic reported as null): %s"
                    % ", ".join(stale))
