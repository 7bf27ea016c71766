"""The benchmark's traffic record is keyed by the code of the kernel sources:
comments and whitespace do not change the key, code does (host only).  A key
that no longer matches makes the benchmark report its traffic as null."""
import bench


def test_code_tokens_drop_comments_keep_code_and_literals():
    a = 'int f(int x) {  // one\n  return x /* two */ + 1;  /* three\n four */ }\nconst char* s = "a // b /* c */";'
    b = 'int f(int x) {\n return x + 1; }   const char* s = "a // b /* c */";'
    assert bench.code_tokens(a) == bench.code_tokens(b)
    assert bench.code_tokens(a) != bench.code_tokens(b.replace("+ 1", "+ 2"))
    assert bench.code_tokens("char c = '/'; // x\nint y;") == "char c = '/'; int y;"
    assert bench.code_tokens('s = "\\" // not a comment";') == 's = "\\" // not a comment";'

