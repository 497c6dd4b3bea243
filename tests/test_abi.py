"""CPU-side checks of the C ABI: the library loads, exports every function
declared in include/*.h, and rejects bad arguments synchronously (no GPU
work is started by these calls)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for hdr in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(hdr).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_ ]*\**\s*\**\s*(sos_[a-z0-9_]+)\s*\(",
                            text, flags=re.M)
    return sorted(set(names))


def test_header_declares_entry_points():
    names = declared_functions()
    for must in ("sos_create", "sos_destroy", "sos_filter", "sos_strerror", "sos_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_2607_23763_amd as P

    lib = P.lib()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_strerror_and_null_handle_rejections():
    import paper_2607_23763_amd as P

    lib = P.lib()
    assert lib.sos_strerror(0) == b"ok"
    assert lib.sos_strerror(-1) == b"invalid argument"
    # every entry point rejects a NULL handle before touching the device
    assert lib.sos_filter(None, None, 1, None, None, 10, None, None, None) == P.SOS_EINVAL
    assert lib.sos_set_tile(None, 64, 32) == P.SOS_EINVAL
    assert lib.sos_get_tile(None, None, None) == P.SOS_EINVAL
    assert lib.sos_set_precision(None, 64) == P.SOS_EINVAL
    assert lib.sos_get_precision(None) == P.SOS_EINVAL
    assert lib.sos_set_algorithm(None, P.SOS_ALG_PH) == P.SOS_EINVAL
    assert lib.sos_get_algorithm(None) == P.SOS_EINVAL
    hdr = open(os.path.join(ROOT, "include", "sosfilt.h")).read()
    for name, val in re.findall(r"(SOS_ALG_[A-Z]+) = (\d+)", hdr):
        assert getattr(P, name) == int(val), name      # binding constants follow the header
    assert lib.sos_set_timeout(None, 1.0) == P.SOS_EINVAL
    assert lib.sos_wall_clock_khz(None) == P.SOS_EINVAL
    assert lib.sos_filter_train_batched(None, 1, 1, 1, 10, None, None, None, None, None, None,
                                        None, None, None, None) == P.SOS_EINVAL
    assert lib.sos_filter_vjp_batched(None, 1, 1, 1, 10, None, None, None, None, None, None, None,
                                      None, None, None, None, None, None) == P.SOS_EINVAL
    assert lib.sos_filter_vjp_batched_sum(None, 1, 1, 1, 10, None, None, None, None, None, None,
                                          None, None, None, None, None, None, None) == P.SOS_EINVAL
    # graph and tuning entry points
    assert lib.sos_graph_create_batched(None, None, 1, 1, 1, 10, None, None, None, None, None,
                                        None, None, None) == P.SOS_EINVAL
    assert lib.sos_graph_launch(None, None) == P.SOS_EINVAL
    assert lib.sos_graph_last_error(None) == P.SOS_EINVAL
    assert lib.sos_graph_destroy(None) == P.SOS_EINVAL
    assert lib.sos_tune_batched(None, 1, 1, 1, 10, None, None, None, None, None, None, None, None,
                                None, 3, None, None, None) == P.SOS_EINVAL
    assert lib.sos_tune_lookup(None, 1, 1, 10, None, None) == P.SOS_EINVAL
    # serving entry points
    assert lib.sos_server_create(None, None, 0, 1) == P.SOS_EINVAL
    assert lib.sos_server_destroy(None) == P.SOS_EINVAL
    assert lib.sos_server_limits(None, None, None, None, None) == P.SOS_EINVAL
    assert lib.sos_stream_open(None, None, 1, None, None) == P.SOS_EINVAL
    assert lib.sos_stream_push(None, 1, None, 10, None, None) == P.SOS_EINVAL
    assert lib.sos_stream_push_many(None, 1, None, None, None, None, None) == P.SOS_EINVAL
    assert lib.sos_stream_wait(None, 1, None) == P.SOS_EINVAL
    assert lib.sos_stream_state(None, 1, None) == P.SOS_EINVAL
    assert lib.sos_stream_close(None, 1) == P.SOS_EINVAL
    assert lib.sos_server_replay(None, 0, None, None, None, None, None, None, None,
                                 None) == P.SOS_EINVAL
    assert lib.sos_filter_batched(None, 1, 1, 1, 10, None, None, None, None, None, None, None,
                                  None, None) == P.SOS_EINVAL
    assert lib.sos_filter_train(None, None, 1, None, None, 10, None, None, None,
                                None) == P.SOS_EINVAL
    assert lib.sos_filter_vjp(None, None, 1, None, None, None, 10, None, None, None, None, None,
                              None) == P.SOS_EINVAL
    assert lib.sos_prepare(None, None, 1, None) == P.SOS_EINVAL
    assert lib.sos_filter_prepared(None, None, None, 10, None, None, None) == P.SOS_EINVAL
    assert lib.sos_bench_copy(None, None, 10, None) == P.SOS_EINVAL
    assert lib.sos_destroy(None) == P.SOS_EINVAL
    assert lib.sos_create(None, 0) == P.SOS_EINVAL
    for name, val in re.findall(r"(SOS_E[A-Z]+) = (-\d+)", hdr):
        assert getattr(P, name) == int(val), name      # status codes too


def test_noalloc_rejects_before_touching_the_device():
    """sos_filter_noalloc checks its arguments and its fixed workspace's
    limits before any HIP call (so these run without a GPU)."""
    import paper_2607_23763_amd as P

    lib = P.lib()
    assert lib.sos_strerror(P.SOS_ELIMIT).startswith(b"beyond the fixed workspace")
    assert lib.sos_filter_noalloc(None, 1, None, None, 10, None, None, None, None) == P.SOS_EINVAL
    assert lib.sos_filter_noalloc(None, 65, None, None, 0, None, None, None, None) == P.SOS_EINVAL
    assert lib.sos_filter_noalloc(None, 0, None, None, -1, None, None, None, None) == P.SOS_EINVAL
    buf = (ctypes.c_float * 16)()
    p = ctypes.cast(buf, ctypes.c_void_p)
    # x and y overlapping without being equal
    assert lib.sos_filter_noalloc(p, 1, p, ctypes.c_void_p(p.value + 4), 8, None, None, None,
                                  None) == P.SOS_EINVAL
    # 2^40 samples at order 16: far beyond the 2^19 group-sections of the workspace
    assert lib.sos_filter_noalloc(p, 8, p, p, 1 << 40, None, None, None, None) == P.SOS_ELIMIT
