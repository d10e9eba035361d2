"""App. F initial-condition smoothing on the GPU (ccmsav_smooth_ic) against
the oracle's relaxation: FP64 to 1e-12, the FP32-transform path to 1e-5,
device and aliased buffers, argument checks, and the context's state left
alone."""
import math
import sys

import numpy as np
import pytest

from oracle import ccmsav_ref as R
from parity_util import rel_linf
from workloads import vesicle_member

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2601_10057_amd import ccmsav as C  # noqa: E402


def note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def sharp_shape(nx, ny, h):
    """A sharp +-1 field: an ellipse with a square notch."""
    x = (np.arange(nx) + 0.5) * h
    y = (np.arange(ny) + 0.5) * h
    X, Y = np.meshgrid(x, y)
    cx, cy = 0.5 * nx * h, 0.5 * ny * h
    inside = np.hypot((X - cx) / (0.35 * nx * h), (Y - cy) / (0.3 * ny * h)) < 1.0
    notch = (np.abs(X - cx - 0.2 * nx * h) < 0.08 * nx * h) & (np.abs(Y - cy) < 0.08 * ny * h)
    return np.where(inside & ~notch, 1.0, -1.0)


@pytest.mark.parametrize("nx,ny", [(64, 64), (256, 256), (128, 64)])
def test_smoothing_matches_oracle_fp64(nx, ny):
    m = vesicle_member(max(nx, ny), 3)
    params = dict(m.params, nx=nx, ny=ny)
    phi0 = np.ascontiguousarray(m.phi0[:ny, :nx])
    psi0 = np.ascontiguousarray(m.psi0[:ny, :nx])
    sharp = sharp_shape(nx, ny, params["h"])
    note(f"smooth fp64 {nx}x{ny}")
    ref = R.smooth_ic(sharp, params["h"], params["eps"], 0.01, 1e-6, 10)
    with C.Context(params, phi0, psi0) as ctx:
        got = ctx.smooth_ic(sharp)
    assert rel_linf(got, ref) <= 1e-12
    assert got.min() >= -1.0 and got.max() <= 1.0
    assert np.abs(got - sharp).max() > 1e-3          # the interface did relax


def test_smoothing_fp32_transforms_and_device_buffers():
    m = vesicle_member(512, 4)
    sharp = sharp_shape(512, 512, m.params["h"])
    ref = R.smooth_ic(sharp, m.params["h"], m.params["eps"], 0.02, 2e-6, 6)
    note("smooth mixed 512")
    with C.Context(m.params, m.phi0, m.psi0, "mixed") as ctx:
        before = ctx.fields()
        got = ctx.smooth_ic(sharp, M=0.02, dt=2e-6, nsteps=6)
        assert rel_linf(got, ref) <= 1e-5
        # device tensors, output aliasing the input
        dev = torch.from_numpy(sharp).cuda()
        C._check(C.load().ccmsav_smooth_ic(ctx._h, 0.02, 2e-6, 6, dev.data_ptr(),
                                           dev.data_ptr()), "smooth")
        assert rel_linf(dev.cpu().numpy(), got) == 0.0
        after = ctx.fields()
        for a, b in zip(before, after):
            assert np.array_equal(a, b)


def test_smoothing_rejects_bad_arguments():
    m = vesicle_member(32, 5)
    sharp = sharp_shape(32, 32, m.params["h"])
    with C.Context(m.params, m.phi0, m.psi0) as ctx:
        for M, dt, n in ((0.0, 1e-6, 1), (0.01, -1.0, 1), (0.01, 1e-6, -1), (math.nan, 1e-6, 1)):
            with pytest.raises(C.CcmsavError) as e:
                ctx.smooth_ic(sharp, M=M, dt=dt, nsteps=n)
            assert e.value.name == "EINVAL"
        # zero steps: only the clipping
        out = ctx.smooth_ic(2.0 * sharp, nsteps=0)
        assert np.array_equal(out, sharp)
