"""The C ABI without a GPU: the built library loads, exports every function
that include/pics.h declares, the Python binding declares a signature for each
of them, the binding's constants equal the header's, and the host-only entry
points (status strings, argument checks before any device work) behave."""
import ctypes
import pathlib
import re

import pytest

from paper_1710_01758_amd import binding as B

ROOT = pathlib.Path(__file__).resolve().parent.parent
HEADER = ROOT / "include" / "pics.h"


def _declared_functions():
    text = HEADER.read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s+\*?([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


def _defines():
    out = {}
    for name, val in re.findall(r"^#define\s+(PICS(?:3D)?_[A-Z0-9_]+)\s+\(?(-?\d+)\)?", HEADER.read_text(), flags=re.M):
        out[name] = int(val)
    return out


@pytest.fixture(scope="module")
def lib():
    path = B.library_path()
    if not path.exists():
        pytest.skip("libpics.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(str(path))


def test_header_parses():
    names = _declared_functions()
    for must in ("pics_create", "build_preconditioner", "apply_A", "apply_Minv", "pcg_solve",
                 "split_bregman_recon", "pics_autotune", "pics_net_loss_grad"):
        assert must in names, must


def test_library_exports_every_declared_function(lib):
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_declares_every_function():
    sig = B.signatures()
    missing = [n for n in _declared_functions() if n not in sig]
    assert not missing, missing


def test_binding_constants_match_header():
    d = _defines()
    assert d["PICS_OK"] == B.PICS_OK
    assert d["PICS_WARN_MAXIT"] == B.PICS_WARN_MAXIT
    assert d["PICS_WARN_FALLBACK"] == B.PICS_WARN_FALLBACK
    for k in ("INVALID", "UNSUPPORTED", "NONFINITE", "BREAKDOWN", "NOT_POSITIVE", "HIP", "STATE"):
        assert d["PICS_ERR_" + k] == getattr(B, "PICS_ERR_" + k)
    assert (d["PICS_MASK_LINES"], d["PICS_MASK_2D"]) == (B.MASK_LINES, B.MASK_2D)
    assert d["PICS_WAVELET_NONE"] == B.WAVELET["none"]
    assert d["PICS_WAVELET_HAAR"] == B.WAVELET["haar"]
    assert d["PICS_WAVELET_DB4"] == B.WAVELET["db4"]
    for k in ("none", "jacobi", "circulant", "learned"):
        assert d["PICS_PRECOND_" + k.upper()] == B.PRECOND[k]
    assert d["PICS_TERM_DATA"] == B.TERM_DATA
    assert d["PICS_TERM_TV"] == B.TERM_TV
    assert d["PICS_TERM_GAMMA"] == B.TERM_GAMMA
    assert d["PICS_TERM_ALL"] == B.TERM_ALL
    assert d["PICS_TERM_WAVELET_EXPLICIT"] == B.TERM_WAVELET_EXPLICIT
    assert d["PICS_OPT_POLL_CHUNK"] == B.OPT_POLL_CHUNK
    assert d["PICS_OPT_GRAPH_BUDGET"] == B.OPT_GRAPH_BUDGET
    assert d["PICS_OPT_COIL_GROUPS"] == B.OPT_COIL_GROUPS
    assert d["PICS_OPT_CONCURRENT_GROUPS"] == B.OPT_CONCURRENT_GROUPS
    assert d["PICS_OPT_COL_TILE"] == B.OPT_COL_TILE
    assert d["PICS_OPT_GRAPH_FIRST_BUDGET"] == B.OPT_GRAPH_FIRST_BUDGET
    assert d["PICS3D_OPT_XCHUNK"] == B.OPT3_XCHUNK
    assert d["PICS_TUNE_FORCE"] == B.TUNE_FORCE
    assert d["PICS_TUNE_NO_WRITE"] == B.TUNE_NO_WRITE


def test_desc_layout_matches_header():
    # pics_desc: m, n, ncoils, mask_kind, wavelet, levels (int32) then mu, lambda, gamma (double)
    assert ctypes.sizeof(B.Desc) == 6 * 4 + 3 * 8
    assert B.Desc.mu.offset == 24


def test_status_strings_and_null_checks(lib):
    lib.pics_status_string.restype = ctypes.c_char_p
    lib.pics_status_string.argtypes = [ctypes.c_int]
    d = _defines()
    seen = set()
    for name, code in d.items():
        if name.startswith("PICS_ERR_") or name.startswith("PICS_WARN_") or name == "PICS_OK":
            s = lib.pics_status_string(code).decode()
            assert s and s not in seen, (name, s)
            seen.add(s)
    # null handles are rejected before any device work
    for fn, nargs in (("pics_destroy", 1), ("apply_A", 4), ("apply_Minv", 3), ("pics_autotune", 2)):
        f = getattr(lib, fn)
        f.restype = ctypes.c_int
        args = [None] + [0] * (nargs - 1)
        assert f(*args) == d["PICS_ERR_INVALID"] or fn == "pics_destroy"
    lib.pics_net_param_count.restype = ctypes.c_int64
    from oracle import learned as OL
    assert lib.pics_net_param_count() == OL.param_count()


def _create(lib, descs, nslices=None):
    """Call pics_create with host placeholder buffers: descriptor checks run
    before any device call, so invalid descriptors are refused on any host."""
    from paper_1710_01758_amd import binding as Bm
    arr = (Bm.Desc * max(1, len(descs)))()
    for i, d in enumerate(descs):
        arr[i] = Bm.Desc(*d)
    h = ctypes.c_void_p()
    dummy = (ctypes.c_uint8 * 16)()
    lib.pics_create.restype = ctypes.c_int
    lib.pics_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32, ctypes.POINTER(Bm.Desc),
                                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    n = len(descs) if nslices is None else nslices
    return lib.pics_create(ctypes.byref(h), n, arr, ctypes.cast(dummy, ctypes.c_void_p),
                           ctypes.cast(dummy, ctypes.c_void_p), None)


GOOD = (256, 256, 12, 0, 2, 3, 1e-3, 4e-3, 4e-3)


@pytest.mark.parametrize("desc,code", [
    ((100, 256, 12, 0, 2, 3, 1e-3, 4e-3, 4e-3), "PICS_ERR_UNSUPPORTED"),   # no FFT plan for 100
    ((256, 2048, 12, 0, 2, 3, 1e-3, 4e-3, 4e-3), "PICS_ERR_UNSUPPORTED"),  # beyond the largest plan
    ((256, 256, 0, 0, 2, 3, 1e-3, 4e-3, 4e-3), "PICS_ERR_INVALID"),        # no coils
    ((256, 256, 12, 7, 2, 3, 1e-3, 4e-3, 4e-3), "PICS_ERR_INVALID"),       # unknown mask kind
    ((256, 256, 12, 0, 5, 3, 1e-3, 4e-3, 4e-3), "PICS_ERR_INVALID"),       # unknown wavelet
    ((64, 64, 4, 0, 2, 7, 1e-3, 4e-3, 4e-3), "PICS_ERR_UNSUPPORTED"),      # 7 levels do not fit 64 x 64
    ((256, 256, 12, 0, 2, 3, -1e-3, 4e-3, 4e-3), "PICS_ERR_INVALID"),      # negative mu
    ((256, 256, 12, 0, 2, 3, 1e-3, float("nan"), 4e-3), "PICS_ERR_INVALID"),  # non-finite lambda
])
def test_create_refuses_invalid_descriptors(lib, desc, code):
    d = _defines()
    assert _create(lib, [GOOD, desc]) == d[code]


def test_create_refuses_empty_batch_and_null_arguments(lib):
    d = _defines()
    assert _create(lib, [GOOD], nslices=0) == d["PICS_ERR_INVALID"]
    lib.pics_create.restype = ctypes.c_int
    assert lib.pics_create(None, 1, None, None, None, None) == d["PICS_ERR_INVALID"]
