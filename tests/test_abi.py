"""Host-side tests of the C ABI: the library loads, exports every declared
entry point, and rejects bad arguments before anything reaches a GPU.

None of these calls enqueues device work (every case returns during argument
checking), so they run without a GPU.
"""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle
from paper_1105_5804_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "swccl.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set()
    for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w]*\s*\**\s*([A-Za-z_]\w*)\s*\(", src, flags=re.M):
        names.add(m.group(1))
    return names


def test_exports_every_declared_symbol():
    L = _lib.lib()
    names = _declared_functions()
    assert {"sw_init", "sw_sweep", "ccl_label", "sw_observables"} <= names
    for n in names:
        assert hasattr(L, n), n
        assert n in _lib.SIGNATURES, n
    hdr = open(os.path.join(ROOT, "include", "swccl.h")).read()
    ver = int(re.search(r"#define SWCCL_ABI_VERSION (\d+)", hdr).group(1))
    assert L.swccl_abi_version() == ver == _lib.ABI_VERSION


def test_status_strings():
    L = _lib.lib()
    for s in range(8):
        assert L.sw_status_string(s) not in (b"", b"unknown status")
    assert L.sw_status_string(99) == b"unknown status"


def test_threshold_matches_oracle():
    L = _lib.lib()
    Ks = [0.0, -3.0, float("inf"), 1e-12, math.log(2.0), math.log1p(math.sqrt(2.0)),
          math.log1p(math.sqrt(3.0))] + list(np.linspace(1e-3, 40, 997))
    for K in Ks:
        assert L.sw_threshold(K) == oracle.threshold(K), K


def _params(W=64, H=64, q=2, kind=0, K=0.88, flags=0, tile_h=0, merge_waves=0):
    return _lib.SwParams(W, H, q, kind, K, 1, 0, flags, tile_h, merge_waves)


def _bufs(spins, ws, nbytes, roots=None, sizes=None):
    return _lib.SwBuffers(spins=spins, workspace=ws, workspace_bytes=nbytes, roots=roots, sizes=sizes)


@pytest.mark.parametrize("kw", [
    dict(W=1), dict(H=1), dict(W=0), dict(W=-5), dict(W=65536, H=32768),
    dict(q=1), dict(q=256), dict(kind=0, q=3), dict(kind=7), dict(K=float("nan")), dict(flags=8),
    dict(tile_h=8), dict(tile_h=48), dict(tile_h=256), dict(tile_h=-64), dict(merge_waves=2),
    dict(merge_waves=32), dict(merge_waves=-8),
])
def test_bad_params_rejected(kw):
    L = _lib.lib()
    p = _params(**kw)
    assert L.sw_workspace_bytes(ctypes.byref(p)) == 0
    h = ctypes.c_void_p()
    buf = _bufs(0x1000, 0x100000, 1 << 30)
    st = L.sw_init(ctypes.byref(h), ctypes.byref(p), ctypes.byref(buf), None)
    assert st in (_lib.SW_ERR_ARG, _lib.SW_ERR_SIZE)


def _few(p, few_b, p_flip, reserved=0):
    p.few_b, p.p_flip, p.reserved = few_b, p_flip, reserved
    return p


@pytest.mark.parametrize("kw,few_b,p_flip,reserved", [
    (dict(q=3, kind=1), 8, 0.5, 0),  # q = 2 only
    (dict(), 8, 1.0, 0),             # p_flip < 1 (else not ergodic)
    (dict(), 8, -0.1, 0),
    (dict(), 8, float("nan"), 0),
    (dict(), -1, 0.5, 0),
    (dict(), 0, 0.0, 1),             # reserved must be 0
])
def test_bad_few_params_rejected(kw, few_b, p_flip, reserved):
    L = _lib.lib()
    p = _few(_params(**kw), few_b, p_flip, reserved)
    assert L.sw_workspace_bytes(ctypes.byref(p)) == 0
    h = ctypes.c_void_p()
    buf = _bufs(0x1000, 0x100000, 1 << 30)
    assert L.sw_init(ctypes.byref(h), ctypes.byref(p), ctypes.byref(buf), None) == _lib.SW_ERR_ARG


def test_few_params_sized_and_kept_out_of_batches():
    """The few-cluster update takes its seed marks (4 B per boundary id) on
    top of the SW workspace; batches refuse it."""
    L = _lib.lib()
    for kind in (0, 1):
        base = L.sw_workspace_bytes(ctypes.byref(_params(W=1000, H=700, kind=kind)))
        few = L.sw_workspace_bytes(ctypes.byref(_few(_params(W=1000, H=700, kind=kind), 16, 0.5)))
        ntiles = -(-1000 // 128) * -(-700 // 64)
        assert few >= base + ntiles * 384 * 4
    assert L.sw_workspace_bytes(ctypes.byref(_few(_params(), 1, 0.0))) > 0
    assert L.sw_workspace_bytes(ctypes.byref(_few(_params(), 10**6, 0.999))) > 0
    P = (_lib.SwParams * 1)(_few(_params(), 8, 0.5))
    assert L.swb_workspace_bytes(P, 1) == 0


def test_good_params_sized():
    L = _lib.lib()
    for W, H in [(2, 2), (64, 64), (4096, 4096), (16384, 16384), (3, 1000)]:
        p = _params(W=W, H=H)
        assert L.sw_workspace_bytes(ctypes.byref(p)) > 0
    big = _params(W=16384, H=16384, q=3, kind=1)
    # codes (2 B/site) dominate; the rest is O(N / tile)
    assert L.sw_workspace_bytes(ctypes.byref(big)) < 16384 * 16384 * 3


def test_thin_lattices_bounded_by_tile_ids():
    """N < 2^31 is not enough: every tile's boundary ids (ntiles x 384) index
    int32 arrays, which bounds very thin lattices."""
    L = _lib.lib()
    for W, H in [(2**30 - 1, 2), (2, 2**30 - 1), (1_000_000_000, 2)]:
        assert W * H < 2**31
        assert L.sw_workspace_bytes(ctypes.byref(_params(W=W, H=H))) == 0, (W, H)
        assert L.ccl_workspace_bytes(W, H, 0) == 0, (W, H)
    for W, H in [(2**22, 2), (2, 2**20), (46340, 46340)]:
        assert L.sw_workspace_bytes(ctypes.byref(_params(W=W, H=H))) > 0, (W, H)
        assert L.ccl_workspace_bytes(W, H, 2) > 0, (W, H)


def test_init_argument_errors():
    L = _lib.lib()
    p = _params()
    need = L.sw_workspace_bytes(ctypes.byref(p))
    h = ctypes.c_void_p()
    assert L.sw_init(None, ctypes.byref(p), None, None) == _lib.SW_ERR_ARG
    buf = _bufs(None, 0x100000, need)
    assert L.sw_init(ctypes.byref(h), ctypes.byref(p), ctypes.byref(buf), None) == _lib.SW_ERR_ARG
    buf = _bufs(0x1000, 0x100000, need - 1)
    assert L.sw_init(ctypes.byref(h), ctypes.byref(p), ctypes.byref(buf), None) == _lib.SW_ERR_WORKSPACE
    buf = _bufs(0x1000, 0x100010, need)
    assert L.sw_init(ctypes.byref(h), ctypes.byref(p), ctypes.byref(buf), None) == _lib.SW_ERR_WORKSPACE
    buf = _bufs(0x1000, None, need)
    assert L.sw_init(ctypes.byref(h), ctypes.byref(p), ctypes.byref(buf), None) == _lib.SW_ERR_WORKSPACE
    # cluster sizes need both output arrays and a larger workspace
    ps = _params(flags=_lib.SW_F_SIZES)
    need_s = L.sw_workspace_bytes(ctypes.byref(ps))
    assert need_s > need
    for r, z in ((None, None), (0x200000, None), (None, 0x300000)):
        buf = _bufs(0x1000, 0x100000, need_s, roots=r, sizes=z)
        assert L.sw_init(ctypes.byref(h), ctypes.byref(ps), ctypes.byref(buf), None) == _lib.SW_ERR_ARG
    buf = _bufs(0x1000, 0x100000, need_s - 1, roots=0x200000, sizes=0x300000)
    assert L.sw_init(ctypes.byref(h), ctypes.byref(ps), ctypes.byref(buf), None) == _lib.SW_ERR_WORKSPACE
    assert L.sw_sweep(None, 1, None) == _lib.SW_ERR_ARG
    assert L.sw_sweep_history(None, 1, 0x1000, None) == _lib.SW_ERR_ARG
    assert L.sw_observables(None, None, None) == _lib.SW_ERR_ARG
    assert L.sw_get_t(None, None) == _lib.SW_ERR_ARG
    assert L.sw_set_t(None, 0) == _lib.SW_ERR_ARG
    assert L.sw_destroy(None) == _lib.SW_ERR_ARG


def test_ccl_argument_errors():
    L = _lib.lib()
    W = H = 100
    need = L.ccl_workspace_bytes(W, H, 0)
    assert need > 0
    assert L.ccl_workspace_bytes(W, H, 3) == 0
    assert L.ccl_workspace_bytes(0, H, 0) == 0
    assert L.ccl_workspace_bytes(65536, 32768, 0) == 0
    assert L.ccl_workspace_bytes(1, 1, 2) > 0
    inp, lab, ws = 0x10000000, 0x20000000, 0x40000000
    call = L.ccl_label
    assert call(None, W, H, 0, lab, None, None, None, ws, need, None) == _lib.SW_ERR_ARG
    assert call(inp, W, H, 0, None, None, None, None, ws, need, None) == _lib.SW_ERR_ARG
    assert call(inp, W, H, 5, lab, None, None, None, ws, need, None) == _lib.SW_ERR_ARG
    assert call(inp, W, H, 0, lab, 0x50000000, None, None, ws, need, None) == _lib.SW_ERR_ARG
    assert call(inp, 0, H, 0, lab, None, None, None, ws, need, None) == _lib.SW_ERR_SIZE
    assert call(inp, W, H, 0, inp + 8, None, None, None, ws, need, None) == _lib.SW_ERR_ARG  # aliasing
    assert call(inp, W, H, 0, lab, None, None, None, ws, 1024, None) == _lib.SW_ERR_WORKSPACE
    assert call(inp, W, H, 0, lab, 0x50000000, 0x60000000, None, ws, need - 1, None) == _lib.SW_ERR_WORKSPACE
    assert call(inp, W, H, 0, lab, None, None, None, None, need, None) == _lib.SW_ERR_WORKSPACE
    assert call(inp, W, H, 0, lab, None, None, None, ws + 4, need, None) == _lib.SW_ERR_WORKSPACE


def test_tile_shapes_sized():
    """Every tile height sizes a workspace; smaller tiles need more boundary ids."""
    L = _lib.lib()
    sizes = {}
    for th in _lib.TILE_HEIGHTS:
        for mw in (0,) + _lib.MERGE_WAVES:
            p = _params(W=1024, H=1024, tile_h=th, merge_waves=mw)
            sizes[th] = L.sw_workspace_bytes(ctypes.byref(p))
            assert sizes[th] > 0
        assert L.ccl_workspace_bytes_tiled(1000, 700, 2, th) > 0
    assert sizes[16] > sizes[32] > sizes[64] > sizes[128]
    assert L.sw_workspace_bytes(ctypes.byref(_params(W=1024, H=1024))) == sizes[64]
    assert L.ccl_workspace_bytes_tiled(1000, 700, 2, 0) == L.ccl_workspace_bytes(1000, 700, 2)
    assert L.ccl_workspace_bytes_tiled(1000, 700, 2, 24) == 0
    inp, lab, ws = 0x10000000, 0x20000000, 0x40000000
    need = L.ccl_workspace_bytes_tiled(100, 100, 0, 32)
    assert L.ccl_label_tiled(inp, 100, 100, 0, 24, 0, lab, None, None, None, ws, need, None) == _lib.SW_ERR_ARG
    assert L.ccl_label_tiled(inp, 100, 100, 0, 32, 3, lab, None, None, None, ws, need, None) == _lib.SW_ERR_ARG
    assert L.ccl_label_tiled(inp, 100, 100, 0, 32, 4, lab, 0x50000000, 0x60000000, None, ws, need - 1,
                             None) == _lib.SW_ERR_WORKSPACE


def test_ccl_noalloc_argument_errors():
    """The allocation-free labeling call refuses bad arguments and shapes whose
    workspace exceeds its static scratch before it touches a device."""
    L = _lib.lib()
    inp, lab = 0x10000000, 0x20000000
    call = L.ccl_label_noalloc
    assert call(None, 64, 64, 0, lab, None, None, None, None) == _lib.SW_ERR_ARG
    assert call(inp, 64, 64, 0, None, None, None, None, None) == _lib.SW_ERR_ARG
    assert call(inp, 64, 64, 3, lab, None, None, None, None) == _lib.SW_ERR_ARG
    assert call(inp, 64, 64, 0, lab, 0x50000000, None, None, None) == _lib.SW_ERR_ARG
    assert call(inp, 0, 64, 0, lab, None, None, None, None) == _lib.SW_ERR_SIZE
    assert call(inp, 64, 64, 0, inp + 8, None, None, None, None) == _lib.SW_ERR_ARG
    # the largest square image with sizes that fits, and the next sizes that do not
    lim = _lib.CCL_NOALLOC_SCRATCH_BYTES
    assert L.ccl_workspace_bytes(2048, 2048, 2) <= lim < L.ccl_workspace_bytes(2560, 2560, 2)
    assert call(inp, 2560, 2560, 2, lab, 0x50000000, 0x60000000, None, None) == _lib.SW_ERR_WORKSPACE
    msg = L.sw_last_error().decode()
    assert str(lim) in msg and str(L.ccl_workspace_bytes(2560, 2560, 2)) in msg
    assert L.ccl_workspace_bytes(8192, 8192, 0) > lim
    assert call(inp, 8192, 8192, 0, lab, None, None, None, None) == _lib.SW_ERR_WORKSPACE


def test_batch_argument_errors():
    L = _lib.lib()
    P = (_lib.SwParams * 3)(_params(), _params(W=100, H=37, q=3, kind=1), _params(W=2, H=2))
    need = L.swb_workspace_bytes(P, 3)
    assert need > 0
    assert L.swb_workspace_bytes(P, 0) == 0
    assert L.swb_workspace_bytes(None, 3) == 0
    bad = (_lib.SwParams * 2)(_params(), _params(W=1))
    assert L.swb_workspace_bytes(bad, 2) == 0
    h = ctypes.c_void_p()
    B = (_lib.SwBuffers * 3)(_bufs(0x1000, None, 0), _bufs(0x2000, None, 0), _bufs(0x3000, None, 0))
    ws = 0x100000
    assert L.swb_init(None, P, B, 3, ws, need, None) == _lib.SW_ERR_ARG
    assert L.swb_init(ctypes.byref(h), P, B, 0, ws, need, None) == _lib.SW_ERR_ARG
    assert L.swb_init(ctypes.byref(h), P, B, 3, ws, need - 1, None) == _lib.SW_ERR_WORKSPACE
    assert L.swb_init(ctypes.byref(h), P, B, 3, ws + 8, need, None) == _lib.SW_ERR_WORKSPACE
    assert L.swb_init(ctypes.byref(h), P, B, 3, None, need, None) == _lib.SW_ERR_WORKSPACE
    B2 = (_lib.SwBuffers * 3)(_bufs(0x1000, None, 0), _bufs(None, None, 0), _bufs(0x3000, None, 0))
    assert L.swb_init(ctypes.byref(h), P, B2, 3, ws, need, None) == _lib.SW_ERR_ARG
    B3 = (_lib.SwBuffers * 3)(_bufs(0x1000, None, 0, roots=0x5000, sizes=0x6000), _bufs(0x2000, None, 0),
                              _bufs(0x3000, None, 0))
    assert L.swb_init(ctypes.byref(h), P, B3, 3, ws, need, None) == _lib.SW_ERR_ARG
    PS = (_lib.SwParams * 1)(_params(flags=_lib.SW_F_SIZES))
    assert L.swb_workspace_bytes(PS, 1) == 0
    assert L.swb_init(ctypes.byref(h), PS, B, 1, ws, need, None) == _lib.SW_ERR_UNSUPPORTED
    PR = (_lib.SwParams * 1)(_params(flags=_lib.SW_F_REVERSE_TILES))  # single lattices only
    assert L.swb_workspace_bytes(PR, 1) == 0
    assert L.swb_init(ctypes.byref(h), PR, B, 1, ws, need, None) == _lib.SW_ERR_UNSUPPORTED
    assert L.sw_workspace_bytes(ctypes.byref(PR[0])) > 0
    assert L.swb_sweep(None, 1, None) == _lib.SW_ERR_ARG
    assert L.swb_sweep_graph(None, 1, None) == _lib.SW_ERR_ARG
    assert L.swb_observables(None, 0, None, None) == _lib.SW_ERR_ARG
    assert L.swb_get_t(None, None) == _lib.SW_ERR_ARG
    assert L.swb_destroy(None) == _lib.SW_ERR_ARG


def test_server_argument_errors():
    L = _lib.lib()
    P = _lib.CclServerParams(2, 1, 8, 2)
    assert L.ccl_server_footprint(100, 50, ctypes.byref(P)) >= 100 * 50 * 13
    assert L.ccl_server_footprint(0, 50, ctypes.byref(P)) == 0
    for bad in (_lib.CclServerParams(3, 1, 8, 2), _lib.CclServerParams(2, 2, 8, 2),
                _lib.CclServerParams(2, 1, 0, 2), _lib.CclServerParams(2, 1, 8, 0),
                _lib.CclServerParams(2, 1, 8, 65)):
        assert L.ccl_server_footprint(100, 50, ctypes.byref(bad)) == 0
        h = ctypes.c_void_p()
        streams = (ctypes.c_void_p * 2)(None, None)
        assert L.ccl_server_create(ctypes.byref(h), ctypes.byref(bad), 0x100000, 1 << 20, streams) == _lib.SW_ERR_ARG
    h = ctypes.c_void_p()
    streams = (ctypes.c_void_p * 2)(None, None)
    assert L.ccl_server_create(None, ctypes.byref(P), 0x100000, 1 << 20, streams) == _lib.SW_ERR_ARG
    assert L.ccl_server_create(ctypes.byref(h), ctypes.byref(P), 0x100000, 1 << 20, None) == _lib.SW_ERR_ARG
    assert L.ccl_server_create(ctypes.byref(h), ctypes.byref(P), 0x100010, 1 << 20, streams) == _lib.SW_ERR_WORKSPACE
    assert L.ccl_server_create(ctypes.byref(h), ctypes.byref(P), None, 1 << 20, streams) == _lib.SW_ERR_WORKSPACE
    slot = ctypes.c_int32()
    assert L.ccl_server_submit(None, 0x1000, 4, 4, 4, 0, ctypes.byref(slot)) == _lib.SW_ERR_ARG
    n = ctypes.c_int32()
    assert L.ccl_server_poll(None, None, None, 0, ctypes.byref(n)) == _lib.SW_ERR_ARG
    assert L.ccl_server_result(None, 0, None, None, None, None) == _lib.SW_ERR_ARG
    assert L.ccl_server_release(None, 0) == _lib.SW_ERR_ARG
    assert L.ccl_server_destroy(None) == _lib.SW_ERR_ARG


def test_missing_library_raises(monkeypatch, tmp_path):
    """Without the built library every call raises: there is no fallback path."""
    import paper_1105_5804_amd as sw

    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "libswccl.so"))
    with pytest.raises(RuntimeError, match="missing"):
        _lib.lib()
    with pytest.raises(RuntimeError, match="missing"):
        sw.threshold(1.0)


@pytest.mark.parametrize("compiler,std,ext", [("gcc", "c99", "c"), ("gcc", "c11", "c"), ("g++", "c++11", "cpp")])
def test_header_compiles_strictly(compiler, std, ext, tmp_path):
    """include/swccl.h is plain C (and C++): no warnings under -Wall -Wextra -Wpedantic."""
    import shutil
    import subprocess

    cc = shutil.which(compiler)
    if cc is None:
        pytest.skip(f"{compiler} not found")
    src = tmp_path / f"use.{ext}"
    src.write_text('#include "swccl.h"\nint main(void) { return (int)sizeof(sw_params) + (int)sizeof(sw_obs); }\n')
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    r = subprocess.run([cc, f"-std={std}", "-Wall", "-Wextra", "-Wpedantic", "-Werror", "-I", inc, "-c", str(src),
                        "-o", str(tmp_path / "use.o")], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stderr


def test_ctypes_layout_matches_header(tmp_path):
    """The binding's structures and constants equal the header's: sizes, field
    offsets and field sizes from a C program built against include/swccl.h."""
    import shutil
    import subprocess

    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("gcc not found")
    structs = {"sw_params": _lib.SwParams, "sw_buffers": _lib.SwBuffers, "sw_obs": _lib.SwObs,
               "ccl_server_params": _lib.CclServerParams, "sw3_params": _lib.Sw3Params}
    consts = ["SW3_REC_ACTIVE", "SW3_REC_NCLUST", "SW3_REC_NSAT", "SW3_REC_COUNTS", "SW3_REC_LEN","SWCCL_ABI_VERSION", "SW_OK", "SW_ERR_ARG", "SW_ERR_SIZE", "SW_ERR_WORKSPACE", "SW_ERR_DEVICE",
              "SW_ERR_STATE", "SW_ERR_UNSUPPORTED", "SW_ERR_HOST_MEMORY", "SW_SPIN_ISING_I8", "SW_SPIN_POTTS_U8",
              "SW_F_KEEP_SPINS", "SW_F_SIZES", "SW_F_REVERSE_TILES", "CCL_BONDS_PERIODIC", "CCL_BONDS_OPEN",
              "CCL_SITES_OPEN", "SW_PHASE_TILE", "SW_PHASE_MERGE", "SW_PHASE_FLIP", "SW_HIST_ACTIVE",
              "SW_HIST_NCLUST", "SW_HIST_MAXCL", "SW_HIST_NSAT", "SW_HIST_COUNTS", "SW_HIST_LEN"]
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "swccl.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("size {cname} %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("field {cname} {f} %zu %zu\\n", offsetof({cname}, {f}), '
                         f"sizeof((({cname} *)0)->{f}));")
    for c in consts:
        lines.append(f'printf("const {c} %lld\\n", (long long)({c}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    exe = str(tmp_path / "layout")
    subprocess.run([cc, "-std=c11", "-I", inc, str(src), "-o", exe], check=True, capture_output=True, timeout=60)
    out = subprocess.run([exe], check=True, capture_output=True, text=True, timeout=60).stdout.split("\n")
    seen = 0
    for line in out:
        w = line.split()
        if not w:
            continue
        if w[0] == "size":
            assert ctypes.sizeof(structs[w[1]]) == int(w[2]), line
        elif w[0] == "field":
            fd = getattr(structs[w[1]], w[2])
            assert (fd.offset, fd.size) == (int(w[3]), int(w[4])), line
        else:
            want = _lib.ABI_VERSION if w[1] == "SWCCL_ABI_VERSION" else getattr(_lib, w[1])
            assert want == int(w[2]), line
        seen += 1
    assert seen == len(structs) + sum(len(p._fields_) for p in structs.values()) + len(consts)


def test_ctypes_signatures_match_prototypes():
    """Every SIGNATURES entry has the header prototype's return type, parameter
    count and parameter types (scalars exactly; struct pointers to the matching
    structure; other pointers as pointers)."""
    hdr = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include",
                            "swccl.h")).read()
    hdr = re.sub(r"/\*.*?\*/", " ", hdr, flags=re.S)
    scalars = {"int32_t": ctypes.c_int32, "sw_status": ctypes.c_int32, "uint32_t": ctypes.c_uint32,
               "uint64_t": ctypes.c_uint64, "size_t": ctypes.c_size_t, "double": ctypes.c_double}
    structs = {"sw_params": _lib.SwParams, "sw_buffers": _lib.SwBuffers, "sw_obs": _lib.SwObs,
               "ccl_server_params": _lib.CclServerParams, "sw3_params": _lib.Sw3Params}

    def agrees(ctype: str, py) -> bool:
        ctype = " ".join(ctype.replace("const", " ").split())
        if "*" not in ctype:
            return py is scalars[ctype]
        base, stars = ctype.replace("*", " ").strip(), ctype.count("*")
        if stars == 1 and base in structs:
            return py is ctypes.POINTER(structs[base])
        if stars == 1 and base in scalars:
            return py in (ctypes.POINTER(scalars[base]), ctypes.c_void_p)
        if stars == 1 and base == "char":
            return py is ctypes.c_char_p
        if stars == 1:  # void * or an opaque handle
            return py is ctypes.c_void_p
        return py is ctypes.POINTER(ctypes.c_void_p)  # an out-pointer to a handle or pointer

    checked = 0
    for name, (res, args) in _lib.SIGNATURES.items():
        m = re.search(r"([\w\s\*]+?)\b" + name + r"\s*\(([^)]*)\)\s*;", hdr)
        assert m, name
        ret = m.group(1).split("\n")[-1]
        assert agrees(ret.replace(name, ""), res), (name, ret)
        params = [p.strip() for p in m.group(2).split(",") if p.strip() and p.strip() != "void"]
        assert len(params) == len(args), (name, params)
        for p, py in zip(params, args):
            ctype = re.sub(r"\b\w+$", "", p.replace("*const*", "**")).strip()  # drop the parameter name
            assert agrees(ctype, py), (name, p, py)
        checked += 1
    assert checked == len(_lib.SIGNATURES)


def _p3(**kw):
    d = dict(Lx=64, Ly=32, Lz=16, q=2, spin_kind=_lib.SW_SPIN_ISING_I8, flags=0, K=0.44, seed=1, stream_id=0,
             reserved=0)
    d.update(kw)
    return _lib.Sw3Params(**d)


def test_cubic_params():
    """sw3_* size good parameters and refuse bad ones before any device work."""
    L = _lib.lib()
    ok = L.sw3_workspace_bytes(ctypes.byref(_p3()))
    assert ok > 64 * 32 * 16 * 3
    for kw in (dict(Lx=0), dict(Ly=-1), dict(Lz=0), dict(Lx=2048, Ly=2048, Lz=512), dict(Lx=1, Ly=1, Lz=2**30),
               dict(q=1), dict(q=256), dict(q=3), dict(spin_kind=7), dict(flags=1), dict(reserved=1),
               dict(K=float("nan"))):
        assert L.sw3_workspace_bytes(ctypes.byref(_p3(**kw))) == 0, kw
    assert L.sw3_workspace_bytes(ctypes.byref(_p3(Lx=1, Ly=1, Lz=1))) > 0
    assert L.sw3_workspace_bytes(ctypes.byref(_p3(q=5, spin_kind=_lib.SW_SPIN_POTTS_U8))) == ok
    # errors found before anything is enqueued (no device pointer is touched)
    p = _p3()
    assert L.sw3_sweep(ctypes.byref(p), None, 0, 1, None, None, None, 256, ok, None) == _lib.SW_ERR_ARG
    assert L.sw3_sweep(ctypes.byref(p), 256, 0, -1, None, None, None, 256, ok, None) == _lib.SW_ERR_ARG
    assert L.sw3_sweep(ctypes.byref(p), 256, 0, 1, None, None, None, None, ok, None) == _lib.SW_ERR_WORKSPACE
    assert L.sw3_sweep(ctypes.byref(p), 256, 0, 1, None, None, None, 256, ok - 1, None) == _lib.SW_ERR_WORKSPACE
    assert L.sw3_sweep(ctypes.byref(p), 256, 0, 1, None, None, None, 257, ok, None) == _lib.SW_ERR_WORKSPACE
    assert L.sw3_sweep(ctypes.byref(p), 256, 2**32 - 2, 3, None, None, None, 256, ok, None) == _lib.SW_ERR_STATE
    assert L.sw3_sweep(ctypes.byref(_p3(Lx=0)), 256, 0, 1, None, None, None, 256, ok, None) == _lib.SW_ERR_SIZE
    assert L.sw3_sweep(ctypes.byref(_p3(q=1)), 256, 0, 1, None, None, None, 256, ok, None) == _lib.SW_ERR_ARG
    assert L.sw3_sweep(None, 256, 0, 1, None, None, None, 256, ok, None) == _lib.SW_ERR_ARG
    assert L.sw3_sweep(ctypes.byref(p), 256, 0, 0, None, None, None, 256, ok, None) == _lib.SW_OK  # nothing to do
    assert L.sw3_init_spins(ctypes.byref(p), None, None) == _lib.SW_ERR_ARG
    assert L.sw3_init_spins(ctypes.byref(_p3(Lz=0)), 256, None) == _lib.SW_ERR_SIZE


def test_ccl3_argument_errors():
    """ccl3_* size good shapes, refuse bad ones and bad arguments before any
    device work."""
    L = _lib.lib()
    ok = L.ccl3_workspace_bytes(64, 32, 16)
    assert ok > 0 and L.ccl3_workspace_bytes(1, 1, 1) > 0
    for shape in ((0, 4, 4), (4, -1, 4), (4, 4, 0), (2048, 2048, 512), (1, 1, 2**30)):
        assert L.ccl3_workspace_bytes(*shape) == 0, shape
    args = dict(bonds=256, labels=256, ws=256, nbytes=ok)

    def call(**kw):
        a = dict(args, **kw)
        return L.ccl3_label(a["bonds"], 64, 32, a.get("Lz", 16), a["labels"], None, a["ws"], a["nbytes"], None)

    assert call(bonds=None) == _lib.SW_ERR_ARG
    assert call(labels=None) == _lib.SW_ERR_ARG
    assert call(ws=None) == _lib.SW_ERR_WORKSPACE
    assert call(nbytes=ok - 1) == _lib.SW_ERR_WORKSPACE
    assert call(ws=260) == _lib.SW_ERR_WORKSPACE
    assert call(Lz=0) == _lib.SW_ERR_SIZE
