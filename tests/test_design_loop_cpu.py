"""Host-side pieces of the inverse-design loop: filter and projection (no GPU needed)."""

import numpy as np
import pytest
import torch
from scipy import ndimage

from paper_2603_24027_amd.optimize import blur3d, gaussian_taps, project


@pytest.mark.parametrize("sigma,shape", [(1.0, (7, 9, 11)), (1.5, (9, 11, 13)), (3.0, (8, 32, 32))])
def test_blur_is_the_truncated_gaussian_filter(sigma, shape):
    # scipy's gaussian_filter with nearest-edge mode and the same truncation radius
    x = np.random.default_rng(1).uniform(size=shape)
    r = int(np.ceil(3 * sigma))
    ref = ndimage.gaussian_filter(x, sigma, mode="nearest", truncate=r / sigma)
    got = blur3d(torch.from_numpy(x), sigma).numpy()
    assert np.abs(got - ref).max() < 1e-12


def test_blur_preserves_constants_and_identity_at_zero_sigma():
    x = torch.full((5, 6, 7), 0.37, dtype=torch.float64)
    assert torch.allclose(blur3d(x, 2.0), x, atol=1e-15)
    y = torch.rand(4, 4, 4, dtype=torch.float64)
    assert torch.equal(blur3d(y, 0.0), y)
    assert abs(float(gaussian_taps(2.5).sum()) - 1.0) < 1e-15


def test_projection_fixed_points_monotone_and_sharp_limit():
    f = torch.linspace(0, 1, 101, dtype=torch.float64)
    for beta in (1.0, 8.0, 64.0):
        p = project(f, beta, 0.5)
        assert abs(float(p[0])) < 1e-15 and abs(float(p[-1]) - 1.0) < 1e-15 and abs(float(p[50]) - 0.5) < 1e-15
        assert torch.all(p[1:] >= p[:-1])
    p = project(f, 1e4, 0.5)
    assert torch.all(p[f < 0.49] < 1e-6) and torch.all(p[f > 0.51] > 1 - 1e-6)


def test_filter_projection_chain_gradient():
    x = torch.rand(3, 4, 5, dtype=torch.float64, requires_grad=True)
    assert torch.autograd.gradcheck(lambda t: project(blur3d(torch.sigmoid(t), 1.2), 6.0), (x,))


def test_subpixel_projection_at_infinite_beta():
    # a planar interface normal to x at f = eta: the projection is the exact fill fraction of each
    # cell (a one-cell ramp), 0 and 1 away from the interface; the gradient does not vanish there
    from paper_2603_24027_amd.optimize import project_subpixel
    x = torch.arange(12, dtype=torch.float64)
    slope = 0.1
    f = (0.5 + slope * (x - 5.3)).view(1, 1, 12).expand(3, 4, 12).clone()   # interface at x = 5.3
    p = project(f, float("inf"), 0.5)
    assert torch.equal(p, project_subpixel(f, 0.5))
    # cell i spans [i - 1/2, i + 1/2]; the filled part is x > 5.3
    want = torch.clamp(x + 0.5 - 5.3, 0.0, 1.0)
    assert torch.allclose(p[1, 2], want, atol=1e-9)
    assert torch.all(p[..., :4] == 0) and torch.all(p[..., 7:] == 1)
    g = torch.zeros_like(f, requires_grad=True)
    (project(f + g, float("inf"), 0.5)[..., 5].sum()).backward()
    assert g.grad[..., 5].abs().min() > 0


def test_beta_schedule_switches_after_forty_iterations():
    from paper_2603_24027_amd.optimize import DesignLoop
    loop = DesignLoop.__new__(DesignLoop)          # the schedule alone (no GPU buffers)
    loop.beta_first, loop.beta_after, loop.switch_at = 1.0, float("inf"), 40
    assert [loop.beta_at(i) for i in (0, 39, 40, 199)] == [1.0, 1.0, float("inf"), float("inf")]
    loop.beta_after = None
    assert loop.beta_at(199) == 1.0
