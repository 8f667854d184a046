"""The source hash that ties a committed profile to the kernel it measured:
comment and whitespace edits keep it, code edits change it."""
import os

from paper_2403_00306_amd import profile_tools as pt


def _hash_with(tmp_path, kernel_src, header_src):
    (tmp_path / "csrc").mkdir(exist_ok=True)
    (tmp_path / "csrc" / "k_tiles.hip").write_text(kernel_src)
    (tmp_path / "csrc" / "pms_internal.h").write_text(header_src)
    old = pt.HERE
    pt.HERE = str(tmp_path)
    try:
        return pt.source_hash("k_tiled")
    finally:
        pt.HERE = old


def test_comments_do_not_matter_code_does(tmp_path):
    base = "int f(int x) {\n  return x + 1; // one\n}\n/* block\n comment */\n"
    hdr = "constexpr int kA = 4;\n"
    h0 = _hash_with(tmp_path, base, hdr)
    h1 = _hash_with(tmp_path, base.replace("// one", "// two words")
                    .replace("block", "other") + "\n\n", hdr)
    assert h0 == h1
    assert _hash_with(tmp_path, base.replace("x + 1", "x + 2"), hdr) != h0
    assert _hash_with(tmp_path, base, "constexpr int kA = 8;\n") != h0


def test_every_listed_kernel_source_exists():
    for k, rel in pt.KERNEL_SOURCES.items():
        assert os.path.exists(os.path.join(pt.HERE, rel)), k
        assert len(pt.source_hash(k)) == 16
