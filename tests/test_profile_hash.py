"""The key under which hardware-counter results are stored
(profile_kernels.source_hash): the code of the stepper sources with comments
and layout removed, and their per-source compiler flags.  An edit of a
comment or of white space keeps the key; an edit of code or of a flag
changes it (bench.py then reports no counter traffic until the counters are
taken again)."""
import os

from paper_1901_06535_amd import build, profile_kernels as pk


def test_code_text_drops_comments_and_layout():
    a = "int x = 1;  // one\n/* block\n comment */ float y=2.0f;\n"
    b = "int x = 1;\n\n\nfloat   y=2.0f;  /* other */\n// trailing\n"
    assert pk.code_text(a) == pk.code_text(b) == "int x = 1; float y=2.0f;"
    assert pk.code_text("a + b") != pk.code_text("a - b")


def test_every_stepper_source_exists():
    for f in pk.STEPPER_SOURCES:
        assert os.path.exists(os.path.join(pk.HERE, "csrc", f)), f


def test_hash_follows_code_and_flags(monkeypatch, tmp_path):
    h0 = pk.source_hash()
    assert h0 == pk.source_hash()
    # a copy of the sources with a comment added and the layout changed
    src = tmp_path / "csrc"
    src.mkdir()
    for f in pk.STEPPER_SOURCES:
        text = open(os.path.join(pk.HERE, "csrc", f), encoding="utf-8").read()
        (src / f).write_text("// a new comment\n" + text.replace("\n", "\n\n"), encoding="utf-8")
    monkeypatch.setattr(pk, "HERE", str(tmp_path))
    assert pk.source_hash() == h0
    # a code change in one source
    f0 = pk.STEPPER_SOURCES[0]
    (src / f0).write_text((src / f0).read_text(encoding="utf-8") + "\nint extra_symbol;\n",
                          encoding="utf-8")
    h1 = pk.source_hash()
    assert h1 != h0
    # a per-source flag on a stepper source
    flags = dict(build.SOURCE_FLAGS)
    flags[pk.STEPPER_SOURCES[1]] = ["-DSOMETHING=1"]
    monkeypatch.setattr(build, "SOURCE_FLAGS", flags)
    assert pk.source_hash() not in (h0, h1)
