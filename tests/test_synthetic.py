"""Input generators (no method arithmetic): the device recipe of the smooth
random velocity equals scipy's Gaussian filter of the same noise, and the
serving mix's gradient-memory rule."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("shape,sigma", [((40, 30, 50), 3.0), ((20, 9), 6.0), ((64, 48), 2.0)])
def test_device_velocity_matches_scipy_filter(shape, sigma):
    from scipy.ndimage import gaussian_filter
    from synthetic import smooth_random_velocity_device
    v = smooth_random_velocity_device(shape, 7, sigma=sigma, vmin=1.5, vmax=4.5, device="cpu").numpy()
    g = torch.Generator(device="cpu")
    g.manual_seed(7)
    noise = torch.randn(shape, generator=g, dtype=torch.float32).numpy().astype(np.float64)
    ref = gaussian_filter(noise, sigma=sigma, mode="reflect", truncate=4.0)
    ref = 1.5 + 3.0 * (ref - ref.min()) / (ref.max() - ref.min())
    assert v.shape == tuple(shape)
    assert abs(v.min() - 1.5) < 1e-12 and abs(v.max() - 4.5) < 1e-12
    assert np.max(np.abs(v - ref)) < 1e-5


def test_serving_gradient_memory_rule():
    from paper_1808_01995_amd.serve import GRADIENT_SHARE, gradient_memory
    budget = 200 << 30
    npts = 1_000_000
    # every forward field fits in the gradient's share: store-all, no budget
    assert gradient_memory(budget, npts, 500, 100) == (-1, 0)
    # too many: automatic revolve pool bounded by the share plus fixed fields
    nck, cap = gradient_memory(budget, npts, 20000, 100)
    assert nck == 0
    fb = npts * 4
    assert cap == budget // GRADIENT_SHARE + 3 * fb + 2 * 20000 * 100 * 4 + (1 << 20)
