"""The kernel-source hash that ties the recorded HBM counters to the kernel:
comments and layout do not change it, code does."""
from paper_2203_10587_amd import profiling as P


def test_strip_comments():
    src = 'int a = 1; // one\n/* two\n lines */ int b = a / 2;  const char* s = "x // y";\n'
    assert P.strip_comments(src) == 'int a = 1; int b = a / 2; const char* s = "x // y";'
    assert P.strip_comments("char c = '\\'';  // q") == "char c = '\\'';"


def test_hash_ignores_comments_not_code(tmp_path, monkeypatch):
    f = tmp_path / "k.hip"
    monkeypatch.setattr(P, "ROOT", str(tmp_path))
    monkeypatch.setattr(P, "KERNEL_SOURCES", ["k.hip"])
    f.write_text("__global__ void k(double* o) { o[0] = 1.0; }  // store\n")
    h0 = P.kernel_hash()
    f.write_text("// a kernel\n__global__ void k(double* o) {\n  o[0] = 1.0;  /* one store */\n}\n")
    assert P.kernel_hash() == h0
    f.write_text("__global__ void k(double* o) { o[0] = 2.0; }\n")
    assert P.kernel_hash() != h0
