"""Host logic of bench.py that needs no GPU: the kernel-source hash that
guards the stored HBM counter figures."""
import bench


def test_code_only_ignores_comments_and_blank_space():
    a = "int f(int x) {\n  // line comment\n  return x + 1; /* block\n comment */\n}\n"
    b = "int f(int x) { return x + 1; }"
    assert bench.code_only(a) == bench.code_only(b)


def test_code_only_keeps_code_changes():
    assert bench.code_only("return x + 1;") != bench.code_only("return x + 2;")
    assert bench.code_only("a[i] = b;  // c") != bench.code_only("a[i] = c;  // b")


def test_stored_traffic_matches_current_sources():
    # the committed counter figures were taken on the current kernel code
    t = bench.stored_traffic("csr_step_laplace2d")
    assert t is not None and 3.0e9 < t < 4.5e9
