"""The C-ABI library loads, exports every declared entry point, and validates
its arguments on the host (no GPU needed for any call made here)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("bpfa.h", "bpfa_serve.h")]


@pytest.fixture(scope="module")
def bpfa():
    from paper_2311_15061_amd import build
    if not os.path.exists(build.LIB_PATH):
        build.build()
    from paper_2311_15061_amd import bpfa as mod
    return mod


def declared_functions():
    names = set()
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(bpfa_[a-z_]+)\s*\(", text))
    return sorted(names)


def test_headers_are_all_listed():
    import glob
    assert sorted(glob.glob(os.path.join(ROOT, "include", "*.h"))) == sorted(HEADERS)


def test_every_declared_symbol_is_exported(bpfa):
    names = declared_functions()
    assert len(names) >= 16
    lib = ctypes.CDLL(bpfa.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    from paper_2311_15061_amd import serve
    assert sorted(bpfa.EXPORTED + serve.EXPORTED) == names


def test_struct_layouts_match_c(bpfa, tmp_path):
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "bpfa_serve.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(bpfa_params),'
                   ' offsetof(bpfa_params, stream), sizeof(bpfa_state_view),'
                   ' offsetof(bpfa_state_view, mem), sizeof(bpfa_stats), offsetof(bpfa_stats, n_sweeps),'
                   ' sizeof(bpfa_server_params), offsetof(bpfa_server_params, device),'
                   ' sizeof(bpfa_serve_result), sizeof(bpfa_serve_stats));'
                   'printf("%zu %zu\\n", sizeof(bpfa_acq_policy), offsetof(bpfa_acq_policy, targeted_share));'
                   'return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    from paper_2311_15061_amd import serve
    want = [ctypes.sizeof(bpfa.Params), bpfa.Params.stream.offset, ctypes.sizeof(bpfa.StateView),
            bpfa.StateView.mem.offset, ctypes.sizeof(bpfa.Stats), bpfa.Stats.n_sweeps.offset,
            ctypes.sizeof(serve.ServerParams), serve.ServerParams.device.offset,
            ctypes.sizeof(serve.ServeResult), ctypes.sizeof(serve.ServeStats),
            ctypes.sizeof(serve.AcqPolicy), serve.AcqPolicy.targeted_share.offset]
    assert got == want


def test_workspace_sizes(bpfa):
    import synth
    sizes = {}
    for name, wl in synth.WORKLOADS.items():
        p = bpfa.make_params(wl.shape, wl.patch, wl.stride, K=wl.K)
        sizes[name] = bpfa.workspace_size(p)
        assert sizes[name] > 0
    assert sizes["lattice64"] < sizes["stem512"] < sizes["stem1024"] < sizes["video256"]
    # every workload fits comfortably in one MI355X's 288 GB of HBM
    assert max(sizes.values()) < 64e9


@pytest.mark.parametrize("kw,status", [
    (dict(shape=(8, 8), patch=(9, 2)), -2),
    (dict(shape=(8, 8), patch=(2, 2), stride=(0, 1)), -2),
    (dict(shape=(10,), patch=(3,), stride=(2,)), -2),        # pixel 9 covered by no patch
    (dict(shape=(8, 8), patch=(2, 2), stride=(3, 1)), -2),   # stride larger than the patch
    (dict(shape=(8, 8), patch=(2, 2), K=0), -2),
    (dict(shape=(8, 8), patch=(2, 2), K=2000), -2),
    (dict(shape=(8, 8), patch=(2, 2), c=0.0), -1),
    (dict(shape=(8, 8), patch=(2, 2), gamma_eps0=float("nan")), -1),
    (dict(shape=(8, 8), patch=(2, 2), problem_id=1 << 24), -1),
])
def test_argument_validation(bpfa, kw, status):
    kw = dict(kw)
    shape, patch = kw.pop("shape"), kw.pop("patch")
    p = bpfa.make_params(shape, patch, **kw)
    with pytest.raises(bpfa.BpfaError) as ei:
        bpfa.workspace_size(p)
    assert ei.value.status == status
    assert bpfa.lib.bpfa_last_error()


def test_bad_ndim_and_null_pointers(bpfa):
    p = bpfa.make_params((8, 8), (2, 2))
    p.ndim = 5
    with pytest.raises(bpfa.BpfaError):
        bpfa.workspace_size(p)
    assert bpfa.lib.bpfa_workspace_size(None, None) == bpfa.EINVAL
    assert bpfa.lib.bpfa_create(None, None, 0, None, None, 0, None) == bpfa.EINVAL
    assert bpfa.lib.bpfa_iterate(None, 1, 1) == bpfa.EINVAL
    assert bpfa.lib.bpfa_sync(None) == bpfa.EINVAL
    assert bpfa.lib.bpfa_set_precision(None, bpfa.BF16) == bpfa.EINVAL
    bpfa.lib.bpfa_destroy(None)


def test_server_rejects_bf16_for_patches_over_256_pixels(bpfa):
    """The BF16 reconstruction's matrix-core tiles hold at most 256 patch pixels;
    a server asking for it with 17 x 17 patches is refused before any device work."""
    import ctypes as ct
    from paper_2311_15061_amd import serve
    p = serve.ServerParams()
    serve.lib.bpfa_server_params_default(ct.byref(p))
    assert p.precision == bpfa.FP32
    p.patch[0], p.patch[1] = 17, 17
    p.precision = bpfa.BF16
    h = ct.c_void_p()
    assert serve.lib.bpfa_server_create(ct.byref(p), ct.byref(h)) == bpfa.ESHAPE
    assert not h.value
