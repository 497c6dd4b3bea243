"""GPU parity of the adjoint (sos_filter_train + sos_filter_vjp and the
autograd Function) against the FP64 oracle's reverse sweep, which is itself
pinned by central finite differences (tests/test_oracle_pins.py)."""
import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2607_23763_amd as P

    P.lib()
    return torch, P


def gpu_vjp(torch, P, sos, x, zi, gy, gzf, tile=None, precision=0):
    h = P.Handle(0, tile=tile, precision=precision)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    y, zf, saved = P.sosfilt_train(d(x), d(sos), d(zi), handle=h)
    gx, gzi, gs = P.sosfilt_vjp(d(sos), d(x), y, saved, d(gy), d(gzf), handle=h)
    torch.cuda.synchronize()
    assert h.last_error() == P.SOS_OK
    return gx.cpu().numpy(), gzi.cpu().numpy(), gs.cpu().numpy()


@pytest.mark.parametrize("tile", [(64, 16), (256, 32), (512, 16)])
@pytest.mark.parametrize("K,n", [(1, 5000), (2, 70001), (4, 1 << 16), (4, 3), (3, 1)])
def test_vjp_matches_oracle(env, K, n, tile):
    torch, P = env
    g = workloads.rng(100 + K + n % 97)
    sos = workloads.random_stable_sos(K, g)
    sos[0] *= 1.25                                       # a0 != 1
    x = workloads.signal(n, seed=7)
    zi = workloads.initial_state(K, g)
    gy = workloads.signal(n, seed=8)
    gzf = workloads.initial_state(K, g, var=1.0)
    gx, gzi, gs = gpu_vjp(torch, P, sos, x, zi, gy, gzf, tile)
    rx, rzi, rs = oracle.sosfilt_vjp(sos, x, zi, gy, gzf)
    print("K", K, "n", n, "tile", tile, rel_l2(gx, rx), rel_l2(gzi, rzi), rel_l2(gs, rs))
    assert rel_l2(gx, rx) <= 1e-5
    assert rel_l2(gzi, rzi) <= 1e-5
    assert rel_l2(gs, rs) <= 1e-4


@pytest.mark.parametrize("precision", [64, 32])
def test_vjp_order16_lightly_damped(env, precision):
    """8 sections, poles at radius 0.995, section 0 scaled to unit white-noise
    gain. The FP64 compute type meets the order-16 bound; FP32 is reported
    beside the FP32 sequential floor of the same reversed-time filter."""
    import scipy.signal

    torch, P = env
    g = workloads.rng(9)
    sos = workloads.random_stable_sos(8, g, r_fixed=0.995)
    h = np.zeros(20000)
    h[0] = 1.0
    hr, _ = oracle.sosfilt(sos, h)
    sos[0, :3] /= np.sqrt(np.sum(hr ** 2))
    n = 1 << 16
    x = workloads.signal(n, seed=10)
    zi = np.zeros((8, 2), np.float32)
    gy = workloads.signal(n, seed=11)
    gx, gzi, gs = gpu_vjp(torch, P, sos, x, zi, gy, np.zeros((8, 2), np.float32),
                          precision=precision)
    rx, rzi, rs = oracle.sosfilt_vjp(sos, x, zi, gy, None)
    # with zero final-state cotangent, gx is the cascade applied to gy in reversed time
    seq = scipy.signal.sosfilt(sos[::-1].astype(np.float32), gy[::-1].astype(np.float32))[::-1]
    print("order16 precision", precision, rel_l2(gx, rx), rel_l2(gzi, rzi), rel_l2(gs, rs),
          "fp32 sequential floor", rel_l2(seq, rx))
    if precision == 64:
        assert rel_l2(gx, rx) <= 1e-5
        assert rel_l2(gzi, rzi) <= 1e-4
        assert rel_l2(gs, rs) <= 1e-4
    else:
        assert np.isfinite(gx).all() and np.isfinite(gs).all()


def test_autograd_function(env):
    torch, P = env
    K, n = 4, 40000
    sos = workloads.sweep_sections(K, "butter")
    x = workloads.signal(n, seed=3)
    zi = workloads.initial_state(K, workloads.rng(4))
    gy = workloads.signal(n, seed=5)
    xt = torch.tensor(x, device="cuda", requires_grad=True)
    st = torch.tensor(sos, device="cuda", requires_grad=True)
    zt = torch.tensor(zi, device="cuda", requires_grad=True)
    y, zf = P.sosfilt_autograd(xt, st, zt)
    (y * torch.tensor(gy, device="cuda")).sum().backward()
    rx, rzi, rs = oracle.sosfilt_vjp(sos, x, zi, gy, None)
    assert rel_l2(xt.grad.cpu().numpy(), rx) <= 1e-5
    assert rel_l2(zt.grad.cpu().numpy(), rzi) <= 1e-5
    assert rel_l2(st.grad.cpu().numpy(), rs) <= 1e-4
