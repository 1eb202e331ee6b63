"""The traffic entries' kernel hash covers code, not comments (CPU only)."""
from paper_1810_11451_amd.probe import traffic


def test_comment_edits_keep_the_hash_code_edits_change_it():
    base = "int f(int x)\n{\n    return x + 1;   // one more\n}\n"
    comment_only = "// new header\nint f(int x)\n{\n\n    return x + 1;   // one more than x\n}\n"
    code_change = "int f(int x)\n{\n    return x + 2;   // one more\n}\n"
    assert traffic._code_only(base) == traffic._code_only(comment_only)
    assert traffic._code_only(base) != traffic._code_only(code_change)


def test_kernel_sha_is_stable_and_keyed():
    assert traffic.kernel_sha("full-width-fp32_3m") == traffic.kernel_sha("uneven-fp32_3m")
    assert traffic.kernel_sha("filter") != traffic.kernel_sha("full-width-fp32_3m")
    assert len(traffic.kernel_sha("filter")) == 16
