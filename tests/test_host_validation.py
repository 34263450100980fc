"""CPU-side checks of argument validation at the C ABI: every call below is
refused (or accepted as a no-op) before the library touches a device, so the
checks run without a GPU. The message of the last failure is kept."""
import ctypes

import pytest


@pytest.fixture(scope="module")
def fp():
    from paper_1903_11749_amd import fppr

    fppr.lib()
    return fppr


def last_error(fp):
    return fp.lib().fppr_last_error().decode()


def test_graph_create_refuses_bad_csr(fp):
    L = fp.lib()
    out = ctypes.c_void_p()
    off = (ctypes.c_uint64 * 2)(0, 0)
    for n, m, ro, mem in ((0, 0, ctypes.cast(off, ctypes.c_void_p), fp.FPPR_MEM_HOST),
                          (0xFFFFFFFF, 0, ctypes.cast(off, ctypes.c_void_p), fp.FPPR_MEM_HOST),
                          (1, 1 << 36, ctypes.cast(off, ctypes.c_void_p), fp.FPPR_MEM_HOST),
                          (1, 0, None, fp.FPPR_MEM_HOST),
                          (1, 0, ctypes.cast(off, ctypes.c_void_p), 7)):
        c = fp.fppr_csr(n, m, ro, None, None, mem)
        assert L.fppr_graph_create(ctypes.byref(c), None, None, ctypes.byref(out)) == fp.FPPR_INVALID_ARGUMENT
        assert out.value is None
        assert last_error(fp)
    c = fp.fppr_csr(1, 5, ctypes.cast(off, ctypes.c_void_p), None, None, fp.FPPR_MEM_HOST)
    assert L.fppr_graph_create(ctypes.byref(c), None, None, ctypes.byref(out)) == fp.FPPR_INVALID_ARGUMENT
    assert "col" in last_error(fp)
    assert L.fppr_graph_create(None, None, None, ctypes.byref(out)) == fp.FPPR_INVALID_ARGUMENT
    one = (ctypes.c_uint64 * 2)(0, 0)
    c = fp.fppr_csr(1, 0, ctypes.cast(one, ctypes.c_void_p), None, None, fp.FPPR_MEM_HOST)
    bad = fp.fppr_graph_opts(0, 5)
    assert L.fppr_graph_create(ctypes.byref(c), ctypes.byref(bad), None, ctypes.byref(out)) == \
        fp.FPPR_INVALID_ARGUMENT
    assert "layout" in last_error(fp)


def test_null_handles(fp):
    L = fp.lib()
    assert L.fppr_graph_destroy(None) == fp.FPPR_OK
    assert L.fppr_batch_destroy(None) == fp.FPPR_OK
    assert L.fppr_server_destroy(None) == fp.FPPR_OK
    assert L.fppr_profile_destroy(None) == fp.FPPR_OK
    assert L.fppr_graph_rebuild(None, None) == fp.FPPR_INVALID_ARGUMENT
    assert L.fppr_graph_set_hub_threshold(None, 8, None) == fp.FPPR_INVALID_ARGUMENT
    assert L.fppr_graph_build_pool(None, None, None) == fp.FPPR_INVALID_ARGUMENT
    assert L.fppr_graph_info(None, None, None, None, None, None) == fp.FPPR_INVALID_ARGUMENT
    lay = ctypes.c_uint32()
    assert L.fppr_graph_layout(None, ctypes.byref(lay)) == fp.FPPR_INVALID_ARGUMENT
    ws = ctypes.c_uint64()
    assert L.fppr_plan(None, None, 1, ctypes.byref(ws)) == fp.FPPR_INVALID_ARGUMENT
    assert L.fppr_run_check(None, None) == fp.FPPR_INVALID_ARGUMENT
    assert L.fppr_profile_read(None, None, None) == fp.FPPR_INVALID_ARGUMENT
    assert L.fppr_profile_read_walk(None, None, None) == fp.FPPR_INVALID_ARGUMENT


def test_batch_refuses_bad_items(fp):
    L = fp.lib()
    ws = ctypes.c_uint64()
    assert L.fppr_batch_plan(None, 0, ctypes.byref(ws)) == fp.FPPR_INVALID_ARGUMENT
    items = (fp.fppr_batch_item * 2)()
    assert L.fppr_batch_plan(items, 2, ctypes.byref(ws)) == fp.FPPR_INVALID_ARGUMENT
    assert "graph is NULL" in last_error(fp)
    out = ctypes.c_void_p()
    assert L.fppr_batch_create(items, 2, None, None, 0, ctypes.byref(out)) == fp.FPPR_INVALID_ARGUMENT
    assert L.fppr_batch_create(items, 2, None, None, 0, None) == fp.FPPR_INVALID_ARGUMENT
    for fn in (L.fppr_batch_launch, L.fppr_batch_check):
        assert fn(None, None) == fp.FPPR_INVALID_ARGUMENT
    assert L.fppr_batch_run(None, None, None, None) == fp.FPPR_INVALID_ARGUMENT
    assert L.fppr_batch_capture(None, None, None) == fp.FPPR_INVALID_ARGUMENT


def test_autotune_and_server_refuse_null(fp):
    L = fp.lib()
    sp = fp.fppr_tune_space()
    res = fp.fppr_tune_result()
    p = fp.make_params(0.15, 16, 1)
    assert L.fppr_autotune(None, ctypes.byref(p), ctypes.byref(sp), ctypes.byref(res), None) == \
        fp.FPPR_INVALID_ARGUMENT
    out = ctypes.c_void_p()
    opts = fp.fppr_server_opts(0, 4, 1 << 20, 1 << 20, 1 << 16, 0)
    assert L.fppr_server_create(None, ctypes.byref(opts), ctypes.byref(out)) == fp.FPPR_INVALID_ARGUMENT
    assert L.fppr_server_create(None, ctypes.byref(opts), None) == fp.FPPR_INVALID_ARGUMENT
    qid = ctypes.c_uint64()
    q = fp.fppr_query()
    assert L.fppr_server_submit(None, ctypes.byref(q), ctypes.byref(qid)) == fp.FPPR_INVALID_ARGUMENT
    assert L.fppr_server_poll(None, 1, None, None, None) == fp.FPPR_INVALID_ARGUMENT
    assert L.fppr_server_wait(None, 1, None, None, None) == fp.FPPR_INVALID_ARGUMENT
    st = fp.fppr_server_counters()
    assert L.fppr_server_stats(None, ctypes.byref(st)) == fp.FPPR_INVALID_ARGUMENT
