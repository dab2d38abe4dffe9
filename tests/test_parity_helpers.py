"""The comparison helpers of the GPU parity tests, exercised on the CPU with
the oracle on both sides: an exact copy passes, and a planted error (in a
copy of the oracle's output) outside the ambiguity zones fails.  This keeps
the band bound and the image-only comparison of batches from being vacuous."""
import math

import numpy as np
import pytest

import parity as P
from paper_2507_16165_amd import inputs


def _render(ref, frame):
    c, s = frame.camera, frame.scene
    cam = ref.camera(c.r, c.incl_deg, c.azim_deg, c.fov_deg, c.width, c.height)
    sc = ref.scene(s.M, r_sky=s.r_sky, disk=s.disk)
    return ref.render(cam, sc)


def _as_gpu(r):
    return {"cls": r.cls.copy(), "b": r.b.copy(), "phi_end": r.phi_end.copy(),
            "exit_dir": r.exit_dir.copy(), "r_hit": r.r_hit.copy()}


@pytest.fixture(scope="module")
def band_frame(ref):
    f = inputs.Frame(inputs.Camera(30.0, 75.0, 20.0, 21.0, 96, 96), inputs.scene_in_m(1.0, (6.0, 20.0)))
    rgba, r = _render(ref, f)
    return f, rgba, r


def test_identical_output_passes(band_frame):
    f, rgba, r = band_frame
    for mode in ("fp64", "fp32"):
        s = P.compare(r, _as_gpu(r), f.scene, mode)
        assert s["band_compared"] > 100
        P.compare_rgba(rgba, r, rgba, r.cls, f.scene, mode)
        assert P.compare_image(rgba, r, rgba, f.scene, mode) > 0.9 * rgba.shape[0] * rgba.shape[1]


def test_band_ray_error_beyond_its_bound_fails(band_frame):
    """A band ray's end azimuth moved by twice its bound fails; by half, passes."""
    f, rgba, r = band_frame
    d = np.abs(r.b - P.B_CRIT)
    k = int(np.nonzero((d > 1e-2) & (d < 0.05) & (r.cls == 0))[0][0])
    lim = 1e-8 + r.b[k] * P.BAND_DRIFT["fp64"] / d[k]
    for scale, ok in ((0.5, True), (2.0, False)):
        g = _as_gpu(r)
        g["phi_end"][k] += scale * lim
        if ok:
            P.compare(r, g, f.scene, "fp64")
        else:
            with pytest.raises(AssertionError):
                P.compare(r, g, f.scene, "fp64")


def test_band_class_flip_fails(band_frame):
    """A band ray 1e-2 M from b_c that changes class fails (it is no longer
    excluded, as all band rays were before)."""
    f, rgba, r = band_frame
    d = np.abs(r.b - P.B_CRIT)
    k = int(np.nonzero((d > 1e-2) & (d < 0.05) & (r.cls == 0))[0][0])
    g = _as_gpu(r)
    g["cls"][k] = 1
    with pytest.raises(AssertionError):
        P.compare(r, g, f.scene, "fp32")


def test_image_comparison_detects_a_wrong_pixel(ref, band_frame):
    """compare_image (colours only): a disk pixel shaded as sky, a sky pixel
    shaded black, and a disk colour 1% off all fail outside the zones."""
    f, rgba, r = band_frame
    H, W = rgba.shape[:2]
    flat = rgba.reshape(-1, 4)
    d = np.abs(r.b - P.B_CRIT)
    clear = d > 0.05
    dsk = np.nonzero(clear & (r.cls == 2) & (r.r_hit > 7.0) & (r.r_hit < 19.0))[0]
    sky = np.nonzero(clear & (r.cls == 0))[0]
    assert dsk.size and sky.size
    for k, val in ((dsk[0], [1.0, 1.0, 1.0, 1.0]), (sky[0], [0.0, 0.0, 0.0, 1.0]),
                   (dsk[1], flat[dsk[1]] * np.array([1.01, 1.01, 1.01, 1.0]))):
        g = flat.copy()
        g[k] = val
        with pytest.raises(AssertionError):
            P.compare_image(rgba, r, g.reshape(H, W, 4), f.scene, "fp32")


def test_image_decode_reads_the_disk_radius(band_frame):
    """The disk radius read back from a disk colour equals the hit radius."""
    f, rgba, r = band_frame
    cls, rr = P._decode_class(rgba, f.scene)
    dsk = r.cls == 2
    np.testing.assert_array_equal(cls[dsk], 2)
    np.testing.assert_allclose(rr[dsk], r.r_hit[dsk], rtol=1e-6)
    assert np.all(cls[r.cls == 1] == 1)
    assert np.all(cls[r.cls == 0] == 0)
