"""Host-side checks of the measurement harness: the committed counter
summaries under profiles/ were taken on the current kernel sources, the bench
finds the records it reports for its default plan, and the source digest
that keys them ignores comments and whitespace."""
import os
import re

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROFILES = os.path.join(ROOT, "profiles")


def test_profiles_name_the_current_sources():
    want = bench.source_digest()
    files = [f for f in sorted(os.listdir(PROFILES)) if f.endswith((".txt", ".md"))]
    assert files
    for f in files:
        text = open(os.path.join(PROFILES, f), encoding="utf-8").read()
        # every summary states the command that made it and its digest
        assert "rocprofv3" in text, f
        named = set(re.findall(r"digest[^\n]*?`([0-9a-f]{16})`", text))
        named |= set(re.findall(r'"source_digest": "([0-9a-f]{16})"', text))
        assert named == {want}, (f, named, want)


def test_bench_finds_its_counter_records():
    # the dominant kernel of every multi-agent plan the tile search chooses
    # between has its traffic and VALU records at the current digest
    for tile in ("16x16-bwd2", "16x16", "32x16", "16x32"):
        for tag in ("traffic", "valu"):
            r = bench.recorded(tag, "k_render_bwd_w", "multi-agent-6x8-640x480", tile)
            assert r is not None, (tag, tile)
            if tag == "traffic":
                assert r["fetch_bytes"] > 0 and r["write_bytes"] > 0
            else:
                assert 0.0 < r["valu_busy_frac"] <= 1.0 and r["valu_insts"] > 0


def test_digest_ignores_comments_and_whitespace():
    a = "int f(int x) {\n  return x + 1;  // one more\n}\n"
    b = "/* the successor */\nint f(int x)\n{ return x + 1; }\n"
    c = "int f(int x) { return x + 2; }\n"
    assert bench._code_only(a) == bench._code_only(b)
    assert bench._code_only(a) != bench._code_only(c)
    # a comment marker inside a string literal is code
    assert bench._code_only('s = "//";') != bench._code_only("s = ;")
