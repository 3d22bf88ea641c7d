"""pic_spectrum_noalloc against pic_spectrum through the C ABI.

The allocation-free entry point sums the spectrum's bins in the library's
static device buffer instead of a buffer allocated per call.  Two calls in a
row, the second on a smaller input (fewer particles, fewer bins, the other
precision), must give what pic_spectrum gives on the same state: bin counts
exactly, weight and spin sums to FP64 summation-order roundoff.  The second
call also shows that nothing of the first call's larger bin range survives in
the buffer.  Sizes beyond the buffer are rejected by the host.
"""

import numpy as np
import pytest

import synth
from paper_2002_02211_amd import spinpic as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    S.load_library()


def _say(*a):
    print("[gpu-case]", *a, flush=True)


def _same(got, want, label):
    c, w, s = got
    c0, w0, s0 = want
    np.testing.assert_array_equal(c, c0, err_msg=label + " counts")
    assert c.sum() > 0, label + ": empty spectrum"
    np.testing.assert_allclose(w, w0, rtol=1e-12, atol=1e-15 * max(1.0, np.abs(w0).max()), err_msg=label)
    np.testing.assert_allclose(s, s0, rtol=1e-12, atol=1e-12 * max(1.0, np.abs(s0).max()), err_msg=label)


def test_noalloc_spectrum_matches_allocating_one_twice():
    spec = synth.preset("small2d")
    state = synth.make_state(spec)
    _say("noalloc spectrum: small2d fp64, 512 bins")
    big = S.Simulation(S.config_from_spec(spec, precision="fp64"), state["particles"], state["fields"])
    big.step(6)
    got = big.spectrum_noalloc(-1, 0.0, 0.2, 512)
    _same(got, big.spectrum(-1, 0.0, 0.2, 512), "first call")
    # a smaller input: a quarter of the particles, FP32, one species, 37 bins
    small_parts = [p[::4].copy() for p in state["particles"]]
    _say("noalloc spectrum: small2d fp32 quarter, 37 bins")
    small = S.Simulation(S.config_from_spec(spec, precision="fp32"), small_parts, state["fields"])
    small.step(3)
    got = small.spectrum_noalloc(0, 0.0, 0.05, 37)
    _same(got, small.spectrum(0, 0.0, 0.05, 37), "second call")
    # and the first context again, after the second call used the buffer
    got = big.spectrum_noalloc(1, 0.0, 1e-4, 1024)
    _same(got, big.spectrum(1, 0.0, 1e-4, 1024), "third call")
    with pytest.raises(S.PicError) as ei:
        big.spectrum_noalloc(-1, 0.0, 1.0, S.PIC_MAX_SPECTRUM_BINS + 1)
    assert ei.value.code == S.PIC_EINVAL
    big.close()
    small.close()
