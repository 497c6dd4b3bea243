"""The cost model of Sec. IV-C (Eqs. (26)-(30)) through the library's C ABI
(host arithmetic: no GPU needed). With the paper's own device budgets
(Table I) it must reproduce Table I's derived rows and Table II's staging
buffer, resident thread blocks, warps, binding budget and hiding-floor mark;
with MI355X's budgets it must give the residency the runtime reports (the GPU
check is in test_gpu_tune.py)."""
import math

import pytest

import paper_2607_23763_amd as P

# Table I: GTX 1070 (Pascal) and RTX 3060 (Ampere)
DEVICES = {
    "GTX 1070": dict(sms=15, smem_per_sm=96 * 1024, smem_per_tb=48 * 1024, regs_per_sm=65536,
                     max_threads_per_sm=2048, max_warps_per_sm=64, max_tbs_per_sm=32,
                     fma_latency=6.0, bandwidth_gbs=256.0),
    "RTX 3060": dict(sms=28, smem_per_sm=100 * 1024, smem_per_tb=48 * 1024, regs_per_sm=65536,
                     max_threads_per_sm=1536, max_warps_per_sm=48, max_tbs_per_sm=16,
                     fma_latency=4.0, bandwidth_gbs=360.0),
}

# Table II: L x N -> (S_buf kB, TBs/SM, warps/SM, regs/thread), pairs GTX / RTX
TABLE_II = {
    (32, 32): (4.2, (23, 16), (23, 16), 72),
    (32, 64): (8.3, (11, 12), (11, 12), 107),
    (32, 128): (16.5, (5, 6), (5, 6), 168),
    (64, 64): (16.6, (5, 6), (10, 12), 105),
}


@pytest.fixture(scope="module")
def lib():
    try:
        return P.lib()
    except OSError as e:
        pytest.skip("library not built: %s" % e)


def paper_device(name):
    d = P.ModelDevice()
    for k, v in DEVICES[name].items():
        setattr(d, k, v)
    d.warp = 32
    d.reg_granule = 8           # 256 registers per warp
    d.issue_rate = 4.0          # four warp schedulers per SM
    d.regs_per_simd_lane = 0
    d.simds = 0
    return d


def test_table_i_roofs_and_hiding_floor(lib):
    """Eq. (28): 32 and 45 GS/s; Eq. (29) with ILP 3: 8 and 6 warps."""
    f = [P.model_floors(paper_device(n)) for n in ("GTX 1070", "RTX 3060")]
    assert [round(x.roof_gss, 6) for x in f] == [32.0, 45.0]
    assert [x.w_min for x in f] == [8, 6]


@pytest.mark.parametrize("shape", sorted(TABLE_II))
def test_table_ii_rows(lib, shape):
    """S_buf = 4 L (N + 1) bytes, resident TBs and warps per SM; shared
    memory binds everywhere except 32 x 32 on the RTX 3060 (TB slots); only
    32 x 128 on the GTX 1070 sits below the hiding floor; registers never
    bind."""
    L, N = shape
    sbuf_kb, tbs, warps, regs = TABLE_II[shape]
    for j, name in enumerate(("GTX 1070", "RTX 3060")):
        c = P.model_config(paper_device(name), L, N, pad=1, regs=regs)
        assert round(c.s_buf / 1000.0, 1) == sbuf_kb
        assert c.tbs_per_sm == tbs[j], (shape, name)
        assert c.warps_per_sm == warps[j], (shape, name)
        tb_cap = shape == (32, 32) and name == "RTX 3060"
        assert c.limit == (P.SOS_MODEL_LIMIT_TBS if tb_cap else P.SOS_MODEL_LIMIT_SMEM)
        assert bool(c.starved) == (shape == (32, 128) and name == "GTX 1070"), (shape, name)
        assert c.feasible


def test_configuration_space_reduces_to_the_four_survivors(lib):
    """Sec. IV-D: N = k L; L below the warp idles lanes; the 48 kB per-TB cap
    excludes L >= 128; residency collapsing to 2-3 TBs per SM (32 x 256)
    excludes large N. Read as: at least 4 resident TBs on both devices."""
    devs = [paper_device(n) for n in DEVICES]
    survivors = []
    for L in (16, 32, 64, 128, 256):
        for k in (1, 2, 4, 8):
            N = k * L
            if N > 256 or L < 32:
                continue
            cs = [P.model_config(d, L, N, pad=1) for d in devs]
            if all(c.feasible and c.tbs_per_sm >= 4 for c in cs):
                survivors.append((L, N))
    assert survivors == [(32, 32), (32, 64), (32, 128), (64, 64)]
    # the excluded neighbours fail for the stated reasons
    assert not P.model_config(devs[0], 128, 128, pad=1).feasible          # per-TB cap
    assert [P.model_config(d, 32, 256, pad=1).tbs_per_sm for d in devs] == [2, 3]


def test_warps_per_sm_is_a_function_of_n_alone(lib):
    """Eq. (30): with shared memory binding, warps per SM ~ S_SM / (128 (N + 1))
    whatever L (here L = 32 and 64 at the same N)."""
    d = paper_device("GTX 1070")
    for N in (64, 128):
        a = P.model_config(d, 32, N, pad=1)
        b = P.model_config(d, 64, N, pad=1)
        est = d.smem_per_sm / (128.0 * (N + 1))
        assert abs(a.warps_per_sm - est) <= 1.0 and abs(b.warps_per_sm - est) <= 2.0


def test_gfx950_budgets(lib):
    """MI355X: 1000 GS/s roof at 8 TB/s; W_min = ceil(1 x 8 / 3) = 3 waves per
    CU; the default tile (512, 64) stages 139264 bytes and keeps one group
    (8 waves) per CU, bound by LDS; (512, 32) at 128 registers keeps two."""
    d = P.model_device_gfx950()
    f = P.model_floors(d)
    assert round(f.roof_gss, 6) == 1000.0 and f.w_min == 3
    c = P.model_config(d, 512, 64, pad=4, regs=248)
    assert c.s_buf == 4 * 512 * 68 and c.tbs_per_sm == 1 and c.warps_per_sm == 8
    assert c.feasible and not c.starved
    c = P.model_config(d, 512, 32, pad=4, regs=128)
    assert c.tbs_per_sm == 2 and c.warps_per_sm == 16
    c = P.model_config(d, 1024, 64, pad=4, regs=248)
    assert not c.feasible                                                  # 278 KB of LDS
    assert math.isclose(d.fp32_tflops, 78.6)


def test_model_rejects_bad_arguments(lib):
    import ctypes

    d = P.model_device_gfx950()
    out = P.ModelConfig()
    assert lib.sos_model_config(None, 64, 16, 4, 0, 3.0, ctypes.byref(out)) == P.SOS_EINVAL
    assert lib.sos_model_config(ctypes.byref(d), 0, 16, 4, 0, 3.0, ctypes.byref(out)) == \
        P.SOS_EINVAL
    assert lib.sos_model_floors(ctypes.byref(d), 0.0, ctypes.byref(P.ModelFloors())) == \
        P.SOS_EINVAL
    assert lib.sos_model_device_gfx950(None) == P.SOS_EINVAL
