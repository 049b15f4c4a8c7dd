"""Static checks that the oracle and the HIP path share no code and that the product
path has no CPU fallback."""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2505_06021_amd")


def py_files(d):
    for dp, _, fs in os.walk(d):
        for f in fs:
            if f.endswith(".py"):
                yield os.path.join(dp, f)


def test_package_never_imports_oracle():
    for f in py_files(PKG):
        src = open(f).read()
        assert not re.search(r"^\s*(from|import)\s+oracle", src, re.M), f


def test_oracle_imports_nothing_from_the_package():
    for f in py_files(os.path.join(ROOT, "oracle")):
        src = open(f).read()
        assert "paper_2505_06021_amd" not in src, f


def test_inputs_module_holds_no_method_step():
    src = open(os.path.join(PKG, "inputs.py")).read()
    for forbidden in ("cholesky", "slogdet", "log1p", "def chi0", "trace"):
        assert forbidden not in src, forbidden


def test_binding_has_no_numpy_compute_fallback():
    src = open(os.path.join(PKG, "rpa.py")).read()
    for forbidden in ("np.linalg", "@ ", "einsum", "import oracle", "matmul"):
        assert forbidden not in src, forbidden
