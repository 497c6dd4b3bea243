"""The no-allocation entry point (sos_filter_noalloc) against the plain
filter's own entry point (sos_filter) on the same inputs, through the C ABI,
two calls in a row (the second smaller, so it runs over the workspace the
first left), and both against the FP64 oracle."""
import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import fp32_bounds, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2607_23763_amd as P

    P.lib()
    return torch, P


def test_noalloc_matches_sos_filter(env):
    torch, P = env
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    err = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    # (K, n, kind): a long random order-16 signal over several groups with a
    # ragged tail, then a shorter order-8 one, then the lightly damped
    # order-16 cascade (the accurate table layout) shorter still
    cases = [(8, (1 << 22) + 12345, "random"), (4, 3 * 8192 + 77, "random"),
             (8, 5000, "damped")]
    for i, (K, n, kind) in enumerate(cases):
        if kind == "damped":
            from tests.test_gpu_forward import lightly_damped_sections

            sos = lightly_damped_sections()
        else:
            sos = workloads.random_stable_sos(K, workloads.rng(700 + i))
        x = workloads.signal(n, seed=710 + i)
        zi = workloads.initial_state(K, workloads.rng(720 + i))
        xd, sd, zid = dev(x), dev(sos), dev(zi)
        print("case", i, "K", K, "n", n, kind, flush=True)
        y_na = torch.empty_like(xd)
        zf_na = torch.empty((K, 2), dtype=torch.float32, device="cuda")
        P.sosfilt_noalloc(xd, sd, y_na, zi=zid, zf=zf_na, err=err)
        y_h, zf_h = P.sosfilt(xd, sd, zid, handle=P.Handle(0))
        torch.cuda.synchronize()
        assert int(err.item()) == 0
        yr, zfr = oracle.sosfilt(sos, x, zi)
        by, bz = fp32_bounds(K, sos, x, zi, yr, zfr)
        a, b = y_na.cpu().numpy(), y_h.cpu().numpy()
        print("  noalloc vs sos_filter", rel_l2(a, b), "vs oracle", rel_l2(a, yr), "bound", by)
        # the same kernels; only the lookback's composition order differs
        assert rel_l2(a, b) <= 1e-6
        assert rel_l2(zf_na.cpu().numpy(), zf_h.cpu().numpy()) <= 1e-6
        assert rel_l2(a, yr) <= by
        assert rel_l2(zf_na.cpu().numpy(), zfr) <= max(bz, 1e-4)


def test_noalloc_degenerate_and_limit(env):
    """n = 0 gives zf = zi, K = 0 copies x, and a request beyond the fixed
    workspace is refused with nothing enqueued."""
    torch, P = env
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    sos = workloads.sweep_sections(2, "butter")
    zi = workloads.initial_state(2, workloads.rng(730))
    x = dev(workloads.signal(1000, seed=731))
    zf = torch.empty((2, 2), dtype=torch.float32, device="cuda")
    P.sosfilt_noalloc(x[:0], dev(sos), torch.empty(0, device="cuda"), zi=dev(zi), zf=zf)
    y = torch.empty_like(x)
    P.sosfilt_noalloc(x, dev(np.zeros((0, 6), np.float32)), y)
    torch.cuda.synchronize()
    assert np.array_equal(zf.cpu().numpy(), zi)
    assert torch.equal(y, x)
    lib = P.lib()
    # in place (x == y), so that only the workspace limit can refuse it
    rc = lib.sos_filter_noalloc(P._p(dev(sos)), 64, P._p(x), P._p(x), 1 << 30, None, None, None,
                                None)
    assert rc == P.SOS_ELIMIT
