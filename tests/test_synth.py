"""The seeded input generator (CPU): determinism per seed, the class
statistics it promises, pure-air end slabs, and the camera and transfer
function helpers the workloads use."""
import numpy as np
import pytest
import torch

from paper_2311_15038_amd import synth


def _small(seed, noise="gauss", n=64):
    return synth.VolumeSpec(n, n, n, seed=seed, noise=noise)


@pytest.mark.parametrize("noise", ["gauss", "poisson64"])
def test_same_seed_same_volume_other_seed_other_volume(noise):
    a = synth.make_volume(_small(11, noise))
    b = synth.make_volume(_small(11, noise))
    c = synth.make_volume(_small(12, noise))
    assert a.dtype == torch.uint16 and a.shape == (64, 64, 64)
    assert torch.equal(a, b)
    assert not torch.equal(a, c)


def test_class_statistics_and_air_end_slabs():
    spec = _small(21, n=96)
    lab = synth.make_labels(spec).numpy()
    v = synth.to_numpy_u16(synth.make_volume(spec)).astype(np.float64)
    assert np.all(lab[:synth.END_SLAB] == 0) and np.all(lab[-synth.END_SLAB:] == 0)
    present = [c for c in range(len(synth.CLASS_MU)) if (lab == c).sum() > 500]
    assert 0 in present and 1 in present and len(present) >= 3
    for c in present:
        x = v[lab == c]
        mu, sd = synth.CLASS_MU[c], synth.CLASS_SIGMA[c]
        # five standard errors of the mean and of the standard deviation (+ rounding)
        assert abs(x.mean() - mu) < 5 * sd / np.sqrt(x.size) + 1.0, (c, x.mean(), mu)
        assert abs(x.std() - sd) < 5 * sd / np.sqrt(2 * x.size) + 1.0, (c, x.std(), sd)


def test_poisson64_noise_is_not_a_comb():
    """64 x Poisson alone would take only multiples of 64; the added Gaussian fills the gaps."""
    v = synth.to_numpy_u16(synth.make_volume(_small(31, "poisson64"))).astype(np.int64)
    assert len(np.unique(v % 64)) == 64


def test_cameras_and_transfer_function():
    cams = synth.turntable_cameras(64, 48, 32, n_views=4)
    c = np.array([32.0, 24.0, 16.0])
    assert cams.shape == (4, 11)
    d = np.linalg.norm(cams[:, 0:3] - c, axis=1)
    assert np.allclose(d, d[0]) and np.allclose(cams[:, 3:6], c) and np.allclose(cams[:, 2], c[2])
    assert np.allclose(cams[:, 6:9], [0, 0, 1]) and np.all(cams[:, 9] == 60.0)
    tf = synth.default_tf()
    assert tf.shape == (256, 4) and tf.dtype == np.float32
    assert np.all(tf[:15, 3] == 0.0) and tf[16, 3] > 0.0       # empty below s = 0.06
    assert np.all(np.diff(tf[:, 3]) >= 0)
