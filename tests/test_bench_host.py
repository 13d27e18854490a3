"""Host logic of bench.py (CPU only): the kernel tag that ties the committed
HBM counter summary to the kernel sources follows the code, not its comments."""
import bench


def test_code_only_strips_comments_keeps_strings():
    src = ('int a = 1; // trailing\n'
           '/* block\n   comment */ const char *s = "x // y /* z */ \\" w";\n'
           '\n'
           '  int b; /* inline */ int c;   \n')
    out = bench._code_only(src)
    assert "trailing" not in out and "block" not in out and "inline" not in out
    assert '"x // y /* z */ \\" w"' in out
    assert out.splitlines() == ['int a = 1;', ' const char *s = "x // y /* z */ \\" w";', '  int b;  int c;']


def test_comment_edits_do_not_change_the_code_text():
    code = "int f(int x)\n{\n    return x + 1;\n}\n"
    commented = "// f adds one\nint f(int x)  // the argument\n{\n    /* the sum */\n    return x + 1;\n}\n\n"
    assert bench._code_only(code) == bench._code_only(commented)
    assert bench._code_only(code) != bench._code_only(code.replace("+ 1", "+ 2"))


def test_kernel_tag_is_stable_hex():
    t = bench.kernel_tag()
    assert len(t) == 16 and int(t, 16) >= 0 and t == bench.kernel_tag()
