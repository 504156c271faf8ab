"""Host-side checks of the C ABI that need no GPU: the library loads and exports
every entry point declared in include/ctm.h."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            text = open(os.path.join(ROOT, "include", h)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            text = re.sub(r"typedef[^;]*;", "", text)
            names |= set(re.findall(r"\b((?:ctm|sur)_[a-z_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("ctm_init", "ctm_sweep", "ctm_energy", "ctm_energy_grad", "ctm_free", "ctm_last_error", "sur_init",
              "sur_predict", "sur_train", "sur_free", "ctm_lbfgs", "ctm_corner_spectra"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2512_14414_amd", "libctm.so"))
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_init_rejects_bad_arguments_without_touching_the_gpu():
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2512_14414_amd", "libctm.so"))
    lib.ctm_init.restype = ctypes.c_int
    lib.ctm_last_error.restype = ctypes.c_char_p
    h = ctypes.c_void_p()
    pat = (ctypes.c_int * 1)(0)
    # chi < D*d is rejected before any device work
    rc = lib.ctm_init(ctypes.byref(h), ctypes.c_void_p(8), 2, 4, 4, 1, 1, pat, 1, 0, None)
    assert rc == -1 and b"chi" in lib.ctm_last_error(None)
    pat2 = (ctypes.c_int * 1)(3)
    rc = lib.ctm_init(ctypes.byref(h), ctypes.c_void_p(8), 2, 2, 8, 1, 1, pat2, 1, 0, None)
    assert rc == -1 and b"pattern" in lib.ctm_last_error(None)


def test_c_program_is_built_next_to_the_library():
    """build() also links a plain C program against the library (run by the GPU tests)."""
    path = os.path.join(ROOT, "paper_2512_14414_amd", "c_abi_check")
    assert os.access(path, os.X_OK)


def test_bench_refuses_more_than_one_gpu():
    """The benchmark has no multi-GPU path: asked for two GPUs it prints one
    JSON line naming the reason and exits with status 2, before any device work."""
    import json
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]
