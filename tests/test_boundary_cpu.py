"""CPU checks of the C-ABI boundary: the library loads, exports every symbol
declared in include/pc.h, sizes workspaces and rejects bad configs (dt above
0.2/w_pe or dx above the Debye length, section II of the paper; null-collision
probability above 0.1).  No compute call is made here (no GPU)."""
import os
import re

import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def native():
    from paper_2202_03215_amd import build, native
    if build.stale():
        build.build()
    return native


def test_every_header_symbol_is_exported(native):
    inc = os.path.join(ROOT, "include")
    declared = set()
    for f in sorted(os.listdir(inc)):
        if f.endswith(".h"):
            text = open(os.path.join(inc, f)).read()
            declared |= set(re.findall(r"^(?:pc_status|void|const char\s*\*)\s*(pc_[a-z0-9_]+)\s*\(", text, re.M))
    assert declared, "no declarations found"
    lib = native.lib()
    for name in declared:
        assert hasattr(lib, name), name
    assert set(native.EXPORTS) <= declared


def test_sizes_scale_with_capacity(native):
    s1 = native.query_sizes(W.small_bounded())
    assert s1.n_nodes == 401 and s1.n_cells == 400
    assert s1.capacity >= 20000 * 1.25
    s2 = native.query_sizes(W.column_50cm())
    assert s2.n_nodes == 5000
    # two ping-pong buffers of 36 bytes per particle per species dominate
    assert s2.workspace_bytes > 4 * 36 * 5_000_000


@pytest.mark.parametrize("bad, status", [
    (dict(dt=1e-9), "PC_ERR_UNSTABLE_CONFIG"),           # dt > 0.2 / w_pe
    (dict(n_cells=40), "PC_ERR_UNSTABLE_CONFIG"),        # dx = 1 mm > lambda_De at 1e15
    (dict(p_torr=40.0), "PC_ERR_UNSTABLE_CONFIG"),       # nu_max dt > 0.1
    (dict(el_p=1.0), "PC_ERR_INVALID_ARG"),
    (dict(n_cells=1), "PC_ERR_INVALID_ARG"),
    (dict(n_cells=20000, L=0.2), "PC_ERR_INVALID_ARG"),  # field solve limited to 8192 nodes
    (dict(ppc=0), "PC_ERR_INVALID_ARG"),
])
def test_bad_configs_rejected(native, bad, status):
    cfg = W.with_(W.column_20cm(), **bad)
    with pytest.raises(native.PcError) as e:
        native.query_sizes(cfg)
    assert status in str(e.value)


def test_batch_sizes_and_rules(native):
    a = W.tiny("periodic", seed=3)
    b = W.tiny("bounded", n_cells=53, L=0.0053, V=5.3, seed=5)
    one = native.query_sizes(a).workspace_bytes + native.query_sizes(b).workspace_bytes
    both = native.query_batch_sizes([a, b])
    assert both > one                       # columns plus the column and item tables
    assert native.query_batch_sizes([a, b, a]) > both
    for bad in (dict(ion_subcycle=7), dict(sort_interval=9), dict(precision="fp32")):
        with pytest.raises(native.PcError) as e:
            native.query_batch_sizes([a, W.with_(b, **bad)])
        assert e.value.status == -1
    with pytest.raises(native.PcError):
        native.query_batch_sizes([a, W.with_(b, dt=1e-6)])   # unstable member
    with pytest.raises(native.PcError):
        native.query_batch_sizes([])


@pytest.mark.parametrize("cells,table_len,ok", [(4096, 120, True), (64, 2, True), (4096, 1024, True),
                                                (4096, 1025, False), (4096, 1, False), (48, 120, False),
                                                (8192, 120, False), (1000, 120, False)])
def test_fluid_config_validation(native, cells, table_len, ok):
    """Fluid columns: power-of-two cell counts in [64, 4096] (cyclic reduction)
    and at most 1024 table rows (the kernels stage the table in LDS); checked
    by the host-side workspace query, no GPU needed."""
    import ctypes as C
    from paper_2202_03215_amd import fluid as FL
    cfg = FL.pc_fluid_config(4, cells, table_len, 0, 1e-9, 0.5, 0.125, 1e6)
    nbytes = C.c_int64(0)
    status = FL._lib().pc_fluid_query(C.byref(cfg), C.byref(nbytes))
    if ok:
        assert status == 0 and nbytes.value > 0
    else:
        assert status != 0
