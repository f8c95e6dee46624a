"""The seeded generators: deterministic per seed and with the statistics the
recipes state (mostly zero motion, horizontal spread above vertical)."""
import numpy as np

from synth import SequenceSpec, blurred_noise, make_config, moving_sequence, qcif_pair


def test_deterministic_per_seed():
    a = qcif_pair(1)
    b = qcif_pair(1)
    c = qcif_pair(2)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)
    assert not np.array_equal(a[0], c[0])
    s1 = make_config(2, frames=4)
    s2 = make_config(2, frames=4)
    np.testing.assert_array_equal(s1, s2)
    assert s1.dtype == np.uint8 and s1.shape == (4, 288, 352)


def test_qcif_truth_statistics():
    zeros, hx, vy = 0, [], []
    n = 0
    for seed in range(1, 41):
        _, _, truth = qcif_pair(seed)
        t = truth.reshape(-1, 2).astype(int)
        zeros += int(((t[:, 0] == 0) & (t[:, 1] == 0)).sum())
        n += len(t)
        nz = t[(t[:, 0] != 0) | (t[:, 1] != 0)]
        hx += list(np.abs(nz[:, 0]))
        vy += list(np.abs(nz[:, 1]))
    frac = zeros / n
    assert 0.6 <= frac <= 0.72  # 0.6 drawn zero, plus Laplace draws that round to 0
    assert np.mean(hx) > 1.5 * np.mean(vy)
    assert max(hx) <= 7 and max(vy) <= 7


def test_blurred_noise_range_and_smoothness():
    rng = np.random.Generator(np.random.PCG64(0))
    x = blurred_noise(rng, 64, 64, 1.5)
    assert x.min() >= 0 and x.max() <= 255
    assert 8 < x.std() < 25
    # Neighbouring pixels are strongly correlated after the blur.
    assert np.corrcoef(x[:, :-1].ravel(), x[:, 1:].ravel())[0, 1] > 0.8


def test_background_pan_is_plus_one():
    seq = moving_sequence(SequenceSpec(352, 288, 3, 0, "uniform6", 6, 9))
    # With no objects, frame t equals frame t-1 shifted one pixel (plus noise).
    cur, ref = seq[2].astype(int), seq[1].astype(int)
    err_pan = np.abs(cur[:, :-1] - ref[:, 1:]).mean()
    err_zero = np.abs(cur - ref).mean()
    assert err_pan < 3.0 < err_zero
