"""The C-ABI library loads and exports every function include/octgs.h
declares, and the binding declares each of them (no GPU work here)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "octgs.h")


def declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^OCTGS_API[^;(]*?\b(octgs_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_entry_points():
    names = declared()
    for must in ("octgs_select_lod", "octgs_decode", "octgs_rasterize_fwd"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2403_17898_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        pytest.fail("liboctgs.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(L.LIB_PATH)
    for name in declared():
        assert hasattr(lib, name), name
    bound = {s[0] for s in L.SIGNATURES}
    assert set(declared()) == bound


def test_host_only_entry_points():
    """Entry points that do host arithmetic only (sizes, validation)."""
    from paper_2403_17898_amd import _lib as L
    lib = L.lib()
    assert lib.octgs_version() >= 1
    assert lib.octgs_select_workspace_bytes(0) > 0
    a = lib.octgs_raster_workspace_bytes(1000, 5000, 128, 128)
    b = lib.octgs_raster_workspace_bytes(2000, 5000, 128, 128)
    assert 0 < a < b
    assert lib.octgs_raster_workspace_bytes(-1, 0, 1, 1) == 0
    # at most 2^24 16x16 tiles per image
    assert lib.octgs_raster_workspace_bytes(0, 0, 65536, 65536) > 0
    assert lib.octgs_raster_workspace_bytes(0, 0, 65536, 65537) == 0
    assert lib.octgs_raster_workspace_bytes(0, 0, 1 << 30, 1 << 30) == 0
    # argument validation fails before any device work
    assert lib.octgs_select_lod(None, None, None, None, None, None, 0, None) == L.OCTGS_EINVAL
    assert lib.octgs_decode(None, None, None, None, None, 0, None, None, 0, None) == L.OCTGS_EINVAL
    assert lib.octgs_decode_explicit(None, None, None, None, None, 0, None, None) == L.OCTGS_EINVAL
    assert lib.octgs_decode_explicit_bwd(None, None, None, None, None, None, 0, None,
                                         None) == L.OCTGS_EINVAL
    assert lib.octgs_prepare_explicit(None, None, None, None, None, None) == L.OCTGS_EINVAL
    assert lib.octgs_strerror(L.OCTGS_ENOSPC) == b"workspace too small"


def test_header_constants_match_binding():
    """Every integer #define and enum value of the header that the binding
    mirrors has the header's value; the rasterizer flags are mirrored."""
    from paper_2403_17898_amd import _lib as L
    src = open(HEADER).read()
    consts = {m.group(1): int(m.group(2)) for m in
              re.finditer(r"^#define\s+(OCTGS_\w+)\s+(\d+)u?\b", src, flags=re.M)}
    consts.update({m.group(1): int(m.group(2)) for m in
                   re.finditer(r"^\s*(OCTGS_\w+)\s*=\s*(-?\d+)", src, flags=re.M)})
    for must in ("OCTGS_RASTER_TRAIN", "OCTGS_RASTER_TILE_ORDER", "OCTGS_EINVAL"):
        assert must in consts and hasattr(L, must), must
    checked = 0
    for name, v in consts.items():
        if hasattr(L, name):
            assert getattr(L, name) == v, name
            checked += 1
    assert checked >= 3


def test_struct_sizes_match_header():
    """ctypes mirrors of the C structs have the C sizes (checked with gcc)."""
    import subprocess
    import tempfile
    from paper_2403_17898_amd import _lib as L
    src = r'''
#include <stdio.h>
#include "octgs.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu\n", sizeof(octgs_camera), sizeof(octgs_anchors),
         sizeof(octgs_mlp), sizeof(octgs_gaussians), sizeof(octgs_raster_params),
         sizeof(octgs_raster_stats));
  printf("%zu %zu %zu %zu\n", sizeof(octgs_explicit), sizeof(octgs_explicit_grads),
         sizeof(octgs_densify_stats), sizeof(octgs_densify_params));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "s.c")
        exe = os.path.join(d, "s")
        open(c, "w").write(src)
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        got = [int(v) for v in subprocess.check_output([exe]).split()]
    want = [ctypes.sizeof(t) for t in (L.Camera, L.Anchors, L.Mlp, L.Gaussians, L.RasterParams,
                                       L.RasterStats, L.Explicit, L.ExplicitGrads,
                                       L.DensifyStats, L.DensifyParams)]
    assert got == want


def test_no_fallback_without_the_library_or_a_gpu(monkeypatch):
    """The product path never falls back: a missing library raises, and so
    does asking for device buffers without a GPU."""
    import torch
    from paper_2403_17898_amd import _lib as L
    monkeypatch.setattr(L, "_lib", None)
    monkeypatch.setattr(L, "LIB_PATH", "/nonexistent/liboctgs.so")
    with pytest.raises(L.OctgsError):
        L.lib()
    if not torch.cuda.is_available():
        import paper_2403_17898_amd as P
        from synth import scenes as S
        sc = S.make_config1()
        with pytest.raises(P.OctgsError):
            P.DeviceScene.from_scene(sc)
