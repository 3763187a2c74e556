"""nvc_select_pixels_noalloc (static device workspace, no allocation) against nvc_select_pixels (caller
workspace): the same multiset, in the same ascending order, bit for bit, on two calls in a row, the second
with a smaller image and batch, so that the first call's counts left in the shared buffer must not leak into
the second's.  Then a call beyond the buffer's maximum is refused on the host."""
import numpy as np
import pytest
import torch

from paper_2506_05930_amd import _lib, api

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _reference(seed, frame, n_pix, batch):
    pix = torch.empty(batch, dtype=torch.int32, device=DEV)
    ws = torch.empty(api.nvc_select_pixels_workspace_bytes(n_pix), dtype=torch.uint8, device=DEV)
    ws.fill_(0x5A)                                   # stale workspace contents must not matter
    api.nvc_select_pixels(seed, frame, n_pix, pix, ws)
    return pix


def test_noalloc_select_pixels_equals_workspace_version():
    cases = [(2, 3, 1920 * 1080, 1 << 18), (7, 11, 4097, 3000)]    # second call: smaller image and batch
    for seed, frame, n_pix, batch in cases:
        print(f"noalloc case seed={seed} frame={frame} n_pix={n_pix} batch={batch}", flush=True)
        got = torch.full((batch,), -7, dtype=torch.int32, device=DEV)
        api.nvc_select_pixels_noalloc(seed, frame, n_pix, got)
        ref = _reference(seed, frame, n_pix, batch)
        torch.cuda.synchronize()
        g, r = got.cpu().numpy(), ref.cpu().numpy()
        assert np.array_equal(g, r), (seed, frame, n_pix, batch)
        assert g.min() >= 0 and g.max() < n_pix and np.all(np.diff(g) >= 0)
    # device counters give the same result as the frame argument
    ctr = api.new_counters(frame=5, step=1)
    a = torch.empty(1000, dtype=torch.int32, device=DEV)
    api.nvc_select_pixels_noalloc(2, 999, 10000, a, ctr=ctr)
    assert torch.equal(a, _reference(2, 5, 10000, 1000))


def test_noalloc_select_pixels_rejects_images_beyond_its_buffer():
    pix = torch.empty(16, dtype=torch.int32, device=DEV)
    with pytest.raises(_lib.NvcError) as e:
        api.nvc_select_pixels_noalloc(2, 0, _lib.NVC_SELECT_PIXELS_NOALLOC_MAX_PIX + 1, pix)
    assert e.value.status == _lib.NVC_ERR_SHAPE
    # the largest image it takes still works
    api.nvc_select_pixels_noalloc(2, 0, _lib.NVC_SELECT_PIXELS_NOALLOC_MAX_PIX, pix)
    torch.cuda.synchronize()
    assert torch.equal(pix, _reference(2, 0, _lib.NVC_SELECT_PIXELS_NOALLOC_MAX_PIX, 16))
