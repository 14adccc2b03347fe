"""Host-side helpers of bench.py (no GPU)."""

import bench


def test_source_code_ignores_comments_and_blank_lines():
    a = "int f(int x)  // the answer\n{\n\n    /* two\n       lines */\n    return x + 1;\n}\n"
    b = "int f(int x)\n{\n    return x + 1; // done\n}"
    assert bench.source_code(a) == bench.source_code(b) == "int f(int x)\n{\n    return x + 1;\n}"
    assert bench.source_code(a) != bench.source_code(b.replace("+ 1", "+ 2"))


def test_counter_summary_requires_matching_geometry(tmp_path):
    p = tmp_path / "c.txt"
    p.write_text("# comment: not a key\nworkload: poly500\nop_tile: 64 8 125\n"
                 "kernel_source_sha256: %s\nop_traffic_bytes_per_dispatch: 123\n" % bench.kernel_source_hash())
    kv, src = bench._counter_summary(str(p), "poly500", [64, 8, 125])
    assert kv["op_traffic_bytes_per_dispatch"] == "123"
    kv, src = bench._counter_summary(str(p), "poly500", [64, 8, 63])
    assert kv is None and src.startswith("stale")
    kv, src = bench._counter_summary(str(p), "poly300", [64, 8, 125])
    assert kv is None
