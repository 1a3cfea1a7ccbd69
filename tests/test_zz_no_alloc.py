"""The frequency mask entry point that allocates nothing (ges_freq_mask_static) gives the bytes of
ges_freq_mask, which takes its scratch from the caller, on two calls in a row (the second smaller, so
the library's scratch array holds the first call's contents when the second starts)."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2402_10128_amd import ges as G

pytestmark = pytest.mark.gpu


def _target(w, h, seed):
    rng = np.random.default_rng(seed)
    # smooth structure plus noise, so the mask has both values
    yy, xx = np.mgrid[0:h, 0:w]
    base = 0.5 + 0.4 * np.sin(xx / 37.0) * np.cos(yy / 23.0)
    img = base[..., None] + 0.1 * rng.standard_normal((h, w, 3))
    return torch.as_tensor(img.astype(np.float32)).cuda()


@pytest.mark.parametrize("omega", [0.75, 0.3])
def test_static_scratch_mask_matches_caller_scratch(omega):
    lib = G.lib()
    for (w, h, seed) in [(1920, 1080, 11), (333, 97, 12)]:
        print(f"[no-alloc mask] {w}x{h} omega={omega}", flush=True)
        tgt = _target(w, h, seed)
        ref = G.ges_freq_mask(tgt, omega)
        out = torch.full((h, w), 7, dtype=torch.uint8, device="cuda")
        st = lib.ges_freq_mask_static(G._ptr(tgt), w, h, C.c_float(omega), G._ptr(out), G._stream())
        assert st == G.GES_OK, lib.ges_last_error()
        torch.cuda.synchronize()
        r, o = ref.cpu().numpy(), out.cpu().numpy()
        assert 0 < int(r.sum()) < r.size, "degenerate mask"
        assert np.array_equal(o, r), f"{int((o != r).sum())} mask bytes differ"


def test_static_scratch_mask_rejects_large_images():
    lib = G.lib()
    tgt = torch.zeros(1, device="cuda")
    out = torch.zeros(1, dtype=torch.uint8, device="cuda")
    assert lib.ges_freq_mask_static(G._ptr(tgt), 16384, 16384, C.c_float(0.75), G._ptr(out), G._stream()) == 2
    assert b"GES_MASK_STATIC_SCRATCH_BYTES" in lib.ges_last_error()
