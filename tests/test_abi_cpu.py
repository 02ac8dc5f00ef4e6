"""The C ABI library is built, loads and exports every symbol the header
declares (no device calls: this runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spgemm.h")
LIB = os.path.join(ROOT, "paper_2206_06611_amd", "libbrmspgemm.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?(?:int|char|void)\s*\*?\s*(\w+)\s*\(", text, flags=re.M)))


def test_header_declares_entry_points():
    names = declared_functions()
    for n in ("spgemm_symbolic", "spgemm_numeric", "spg_create", "spg_destroy", "spg_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        import importlib.util
        spec = importlib.util.spec_from_file_location(
            "_brm_build", os.path.join(ROOT, "paper_2206_06611_amd", "build.py"))
        mod = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(mod)
        mod.build()
    lib = ctypes.CDLL(LIB)
    for n in declared_functions():
        assert hasattr(lib, n), n


def test_binding_lists_every_declared_symbol():
    import importlib.util
    spec = importlib.util.spec_from_file_location("_pkgsrc", os.path.join(ROOT, "paper_2206_06611_amd", "__init__.py"))
    src = open(spec.origin).read()
    for n in declared_functions():
        assert f'"{n}"' in src, n


def test_null_arguments_are_rejected_without_a_device():
    lib = ctypes.CDLL(LIB)
    lib.spg_create.argtypes = [ctypes.c_void_p, ctypes.c_int]
    assert lib.spg_create(None, 0) == -1          # SPG_ERR_ARG
    lib.spg_destroy.argtypes = [ctypes.c_void_p]
    assert lib.spg_destroy(None) == -1
    lib.spgemm_symbolic.argtypes = [ctypes.c_void_p] * 6
    assert lib.spgemm_symbolic(None, None, None, None, None, None) == -1
