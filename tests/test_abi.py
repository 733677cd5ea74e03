"""The C-ABI library loads on the host and exports every symbol the header
declares; the Python binding covers the whole header.  No GPU work."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "qb.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qb_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_2502_13947_amd import qb
    assert os.path.exists(qb.LIB_PATH), "build() must have produced libqb.so"
    L = ctypes.CDLL(qb.LIB_PATH)
    names = header_functions()
    assert len(names) >= 25
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_header():
    from paper_2502_13947_amd import qb
    assert set(header_functions()) == set(qb.SIGNATURES)


def test_host_only_calls_work_without_gpu():
    from paper_2502_13947_amd import qb
    L = qb.lib()
    assert L.qb_status_str(-2).decode() == "Q is not symmetric"
    assert qb.mutation_rate(15) == 0.0
    assert qb.threshold_table(2, 4, 10.0, 0.0)[1].max() == 0
    # argument errors are reported before any device work
    assert L.qb_init_solutions(0, 1, 0, None, None) == -1
    assert L.qb_threshold_table(0, 10, 1.0, 1.0, None) == -1


def test_product_path_does_not_touch_the_oracle():
    pkg = os.path.join(ROOT, "paper_2502_13947_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src, f
                assert "qbo_" not in src, f
