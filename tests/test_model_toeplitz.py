"""The whole-cascade block-Toeplitz algorithm (tests/toeplitz_model.py)
against the FP64 oracle, on the CPU: its algebra in FP64 (every column, tile,
group and chunk boundary, ragged ends, initial states, random lookback
lengths, with and without the power-of-two state scaling), and its FP32
accuracy on the cascades the GPU path takes."""
import numpy as np
import pytest

import oracle
import workloads
from tests import toeplitz_model as TM
from tests.gpu_util import fp32_floor, rel_l2

SMALL = dict(M=8, TC=4, NT=4, NG=2)        # 128-sample groups, 256-sample chunks


@pytest.mark.parametrize("ng", [2, 4])
@pytest.mark.parametrize("K", [1, 3, 8])
@pytest.mark.parametrize("n", [1, 7, 8, 127, 128, 256, 1000, 2049])
def test_fp64_model_matches_oracle(K, n, ng):
    """Every column, tile, group and chunk boundary of the small shape, with
    chunks of 2 and 4 groups (the chunk map H = G^NG and its powers)."""
    sos = workloads.sweep_sections(K, "random")
    x = workloads.signal(n, 3 + n)
    zi = workloads.initial_state(K, workloads.rng(K))
    ref, zref = oracle.sosfilt(sos.astype(np.float64), x.astype(np.float64), zi.astype(np.float64))
    y, zf = TM.run(sos, x, zi, **dict(SMALL, NG=ng), rng=np.random.default_rng(n))
    assert rel_l2(y, ref) < 1e-10
    assert rel_l2(zf, np.asarray(zref).reshape(K, 2)) < 1e-10


def test_scaling_changes_nothing_in_fp64():
    """D is a power of two per state entry: the scaled and unscaled forms
    agree to rounding, and the scaled form's tables are O(1)."""
    sos = workloads.random_stable_sos(8, workloads.rng(9), r_fixed=0.995)
    sos[0, :3] *= 1e-6          # a first section scaled far down: huge later states
    x = workloads.signal(3000, 1)
    y1, z1 = TM.run(sos, x, **SMALL)
    y2, z2 = TM.run(sos, x, **SMALL, balanced=False)
    assert rel_l2(y1, y2) < 1e-9 and rel_l2(z1, z2) < 1e-9
    phi, g, c, d = TM.cascade_ss(sos)
    D = TM.balance(phi, g, c, 64)
    assert np.all(np.log2(D) == np.rint(np.log2(D)))
    assert np.max(np.abs(g)) > 1e3 * np.max(np.abs(g / D))


def test_impulse_response_is_the_cascade():
    """T's first column is the cascade's impulse response (h[0] = d,
    h[i] = c Phi^(i-1) gamma), which the oracle gives independently."""
    sos = workloads.butterworth_sos(6)
    phi, g, c, d = TM.cascade_ss(sos)
    h = [d] + [c @ np.linalg.matrix_power(phi, i - 1) @ g for i in range(1, 64)]
    imp = np.zeros(64)
    imp[0] = 1.0
    ref, _ = oracle.sosfilt(sos.astype(np.float64), imp)
    assert np.max(np.abs(np.array(h) - ref)) < 1e-12


@pytest.mark.parametrize("kind,K,bound,ng", [("butter", 8, 1e-6, 8), ("random", 8, 1e-6, 8),
                                             ("butter", 4, 1e-6, 8), ("random", 8, 1e-6, 4),
                                             ("random", 8, 1e-6, 2), ("butter", 8, 1e-6, 2)])
def test_fp32_accuracy_at_the_kernel_shape(kind, K, bound, ng):
    """FP32 with the kernel's shape (64-sample columns, 16 x 16 tiles and
    groups, chunks of 8, 4 or 2 groups): rel-L2 far inside the north-star
    bounds."""
    sos = workloads.sweep_sections(K, kind)
    x = workloads.signal(2 * 131072 + 999, 5)
    ref, _ = oracle.sosfilt(sos.astype(np.float64), x.astype(np.float64))
    y, _ = TM.run(sos, x, dtype=np.float32, NG=ng)
    assert rel_l2(y, ref) < bound


def test_fp32_near_the_unit_circle_is_a_sequential_filter():
    """Poles at radius 0.995: the FP32 form stays within 3x the error of a
    sequential FP32 cascade on the same input (which the GPU test bounds at
    10x), and within the order-16 bound."""
    sos = workloads.random_stable_sos(8, workloads.rng(9), r_fixed=0.995)
    imp = np.zeros(40000)
    imp[0] = 1.0
    hr, _ = oracle.sosfilt(sos.astype(np.float64), imp)
    sos[0, :3] /= np.sqrt(np.sum(hr ** 2))
    sos = sos.astype(np.float32)
    x = workloads.signal(131072 + 77, 21)
    ref, _ = oracle.sosfilt(sos.astype(np.float64), x.astype(np.float64))
    y, _ = TM.run(sos, x, dtype=np.float32)
    e, floor = rel_l2(y, ref), fp32_floor(sos, x, None, ref)
    assert e < 3 * floor and e < 1e-4, (e, floor)
