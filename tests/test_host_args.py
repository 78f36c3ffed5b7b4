"""Host side of the C ABI, without a GPU: every entry point rejects missing
pointers and negative sizes before it enqueues anything, zero-sized work
returns OK without a launch, and the workspace views of the rasterizer lie
inside the workspace that octgs_raster_workspace_bytes sizes."""

import ctypes

import pytest

from paper_2403_17898_amd import _lib as L


@pytest.fixture(scope="module")
def lib():
    return L.lib()


def test_missing_pointers_rejected(lib):
    E = L.OCTGS_EINVAL
    calls = {
        "octgs_prepare_anchors": (None,) * 5,
        "octgs_select_lod_noalloc": (None,) * 6,
        "octgs_rasterize_fwd": (None, None, None, 0, None, None, None, None, None, 0, None, None),
        "octgs_rasterize_bwd": (None, None, None, 0, None, None, None, None, None, 0, None, None),
        "octgs_decode_bwd": (None, None, None, None, None, None, 0, None, None, None, 0, None),
        "octgs_decode_bwd_rows": (None, None, None, None, None, None, 0, None, 0, None),
        "octgs_decode_bwd_apply": (None, None, None, None, 0, None, None, None, 0, None),
        "octgs_l1_loss_grad": (None, None, 16, 1.0, None, None, None),
        "octgs_photometric_loss_grad": (None, None, 1, 8, 8, 0.8, 0.2, None, None, None, 0, None),
        "octgs_volume_loss_grad": (None, 0.01, None, None, None),
        "octgs_adam_step": (None, None, None, None, 16, 1e-3, 0.9, 0.999, 1e-8, 1, None),
        "octgs_adam_step_many": (2, None, None, None, None, None, 1e-3, 0.9, 0.999, 1e-8, 1, None),
        "octgs_anchor_weights": (None, None, 10, 100, None, None),
        "octgs_skip_features": (None, None, None, None, 100, None, None),
        "octgs_skip_predict": (None, None, None, 0.0, None, None, 100, None, None, None, None, 0,
                               None),
        "octgs_skip_train_grad": (None, None, None, None, 64, 0, 1.0, None, None, None, 0, None),
        "octgs_densify_accumulate": (None, None, 0, None, 0, None, None, 10, None, None),
        "octgs_densify_decide": (None,) * 8,
        "octgs_raster_views": (None, 100, 100, 64, 64, None, None, None, None),
    }
    for name, args in calls.items():
        assert getattr(lib, name)(*args) == E, name


def test_invalid_sizes_rejected(lib):
    E = L.OCTGS_EINVAL
    buf = ctypes.c_void_p(1 << 40)  # never dereferenced: validation fails first
    assert lib.octgs_l1_loss_grad(buf, buf, -1, 1.0, buf, buf, None) == E
    assert lib.octgs_adam_step(buf, buf, buf, buf, -1, 1e-3, 0.9, 0.999, 1e-8, 1, None) == E
    # Adam's step counter starts at 1 (bias corrections 1 / (1 - beta^t))
    assert lib.octgs_adam_step(buf, buf, buf, buf, 16, 1e-3, 0.9, 0.999, 1e-8, 0, None) == E
    assert lib.octgs_adam_step_many(-1, None, None, None, None, None, 1e-3, 0.9, 0.999, 1e-8, 1,
                                    None) == E
    assert lib.octgs_photometric_loss_grad(buf, buf, -1, 8, 8, 0.8, 0.2, buf, buf, buf, 0,
                                           None) == E
    assert lib.octgs_photometric_loss_grad(buf, buf, 1, -8, 8, 0.8, 0.2, buf, buf, buf, 0,
                                           None) == E
    # negative loss weights, and more planes than the grid's z extent holds
    assert lib.octgs_photometric_loss_grad(buf, buf, 1, 8, 8, -0.8, 0.2, buf, buf, buf, 1 << 30,
                                           None) == E
    assert lib.octgs_photometric_loss_grad(buf, buf, 65536, 8, 8, 0.8, 0.2, buf, buf, buf,
                                           1 << 40, None) == E
    assert lib.octgs_anchor_weights(buf, buf, 0, 100, buf, None) == E
    assert lib.octgs_anchor_weights(buf, buf, 10, -1, buf, None) == E
    assert lib.octgs_raster_views(buf, 100, 100, 0, 64, None, None, None, None) == E
    assert lib.octgs_raster_views(buf, -1, 100, 64, 64, None, None, None, None) == E


def test_workspace_too_small(lib):
    """A photometric call with SSIM needs its three derivative maps."""
    buf = ctypes.c_void_p(1 << 40)
    need = lib.octgs_photometric_workspace_bytes(3, 64, 64)
    assert need >= 3 * 3 * 64 * 64 * 4
    assert lib.octgs_photometric_loss_grad(buf, buf, 3, 64, 64, 0.8, 0.2, buf, buf, buf, need - 1,
                                           None) == L.OCTGS_ENOSPC


def test_zero_sized_work_is_a_no_op(lib):
    """Nothing to do returns OK before any launch (no GPU here)."""
    OK = L.OCTGS_OK
    assert lib.octgs_l1_loss_grad(None, None, 0, 1.0, None, None, None) == OK
    assert lib.octgs_adam_step(None, None, None, None, 0, 1e-3, 0.9, 0.999, 1e-8, 1, None) == OK
    assert lib.octgs_adam_step_many(0, None, None, None, None, None, 1e-3, 0.9, 0.999, 1e-8, 1,
                                    None) == OK
    assert lib.octgs_photometric_loss_grad(None, None, 0, 8, 8, 0.8, 0.2, None, None, None, 0,
                                           None) == OK
    # SSIM weight 0 is the L1 term alone and needs no workspace
    assert lib.octgs_photometric_workspace_bytes(0, 8, 8) > 0
    assert lib.octgs_photometric_workspace_bytes(-1, 8, 8) == 0


@pytest.mark.parametrize("gcap,pcap,W,H", [(1, 1, 1, 1), (1000, 5000, 128, 128),
                                           (270000, 1 << 21, 1920, 1080),
                                           (5, 7, 4096 + 3, 17)])
def test_raster_views_inside_workspace(lib, gcap, pcap, W, H):
    """The stats header, the sorted (tile, slot) lists and the tile ranges
    that octgs_raster_views returns are 256-byte aligned, do not overlap and
    end inside octgs_raster_workspace_bytes from the base (pointer arithmetic
    only: the base is a made-up address that is never read)."""
    base = 1 << 40
    size = lib.octgs_raster_workspace_bytes(gcap, pcap, W, H)
    assert size > 0
    out = [ctypes.c_void_p() for _ in range(4)]
    st = lib.octgs_raster_views(ctypes.c_void_p(base), gcap, pcap, W, H,
                                *[ctypes.byref(o) for o in out])
    assert st == L.OCTGS_OK
    stats, tile, slot, ranges = (o.value for o in out)
    tiles = ((W + 15) // 16) * ((H + 15) // 16)
    spans = [(stats, ctypes.sizeof(L.RasterStats)), (tile, 4 * pcap), (slot, 4 * pcap),
             (ranges, 8 * tiles)]
    for p, n in spans:
        assert p is not None and (p - base) % 256 == 0
        assert base <= p and p + n <= base + size
    spans.sort()
    for (p0, n0), (p1, _) in zip(spans, spans[1:]):
        assert p0 + n0 <= p1
    # the views are the same for the same shape, and only the base moves them
    out2 = [ctypes.c_void_p() for _ in range(4)]
    assert lib.octgs_raster_views(ctypes.c_void_p(base + (1 << 20)), gcap, pcap, W, H,
                                  *[ctypes.byref(o) for o in out2]) == L.OCTGS_OK
    assert [o.value - (1 << 20) for o in out2] == [stats, tile, slot, ranges]
