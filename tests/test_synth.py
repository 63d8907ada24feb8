"""Synthetic ALMA-shaped inputs: sizes, reproducibility, Nyquist sampling."""
import numpy as np
import pytest

from paper_1703_02920_amd import synth


@pytest.mark.parametrize("c,n_bl,z", [(1, 190, 5130), (2, 780, 99840), (3, 1225, 999600),
                                      (5, 1770, 5000250)])
def test_baseline_and_visibility_counts(c, n_bl, z):
    p = synth._CFG[c]
    rng = synth._rngs(c)[0]
    pos = synth.antenna_layout(rng, p["n_ant"], p["diam"])
    bl, _, _ = synth.baselines(pos)
    assert bl.shape[0] == n_bl
    assert bl.shape[0] * p["n_int"] == z
    # antennas inside the disk and at least 15 m apart
    assert np.all(np.hypot(pos[:, 0], pos[:, 1]) <= p["diam"] / 2)
    d = np.hypot(bl[:, 0], bl[:, 1])
    assert d.min() >= synth.MIN_SPACING_M


def test_c4_slot_count_and_channel_sizes():
    ds = synth.make_config(4, channels=3)
    assert synth._CFG[4]["n_int"] * 990 == 300960
    assert ds.n_chan == 3
    for ch in ds.channels:
        assert 20000 <= ch.nvis <= 300000
    # wavelength steps 0.1 % per channel; beam scales with wavelength
    lam = [ch.wavelength for ch in ds.channels]
    assert np.allclose(np.diff(np.log(lam)), np.log(1.001))
    assert np.allclose([ch.fwhm / ch.wavelength for ch in ds.channels], ds.channels[0].fwhm / lam[0])


def test_reproducible_and_nyquist():
    a = synth.make_config(1)
    b = synth.make_config(1)
    assert np.array_equal(a.channels[0].vis, b.channels[0].vis)
    assert np.array_equal(a.channels[0].u, b.channels[0].u)
    ch = a.channels[0]
    umax = max(np.abs(ch.u).max(), np.abs(ch.v).max())
    assert 1.0 / a.cell >= 2 * umax
    assert a.sky.max() == pytest.approx(1.0)
    assert ch.vis.dtype == np.complex64 and ch.w.dtype == np.float32 and ch.u.dtype == np.float64


def test_beam_fwhm_scaling():
    """21 arcsec at 300 GHz (Sec. 2.4) -> 27.32 arcsec at 1.3 mm."""
    assert synth.beam_fwhm(synth.C_LIGHT / 300e9) / synth.ARCSEC == pytest.approx(21.0)
    assert synth.beam_fwhm(1.3e-3) / synth.ARCSEC == pytest.approx(27.3189, rel=1e-4)
