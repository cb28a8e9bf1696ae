"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/dr.h, and rejects invalid input (validation runs before
any HIP call, so these run on a CPU-only machine)."""
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2305_07030_amd import build as B
from paper_2305_07030_amd import dr
from paper_2305_07030_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "dr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\**\s*(dr_\w+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if B.stale():
        B.build()
    return dr.load()


def test_exports_every_declared_function(lib):
    names = header_functions()
    assert len(names) >= 11
    assert set(names) == set(dr.EXPORTS)
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\sT\s(\w+)$", out, flags=re.M))
    for n in names:
        assert n in exported, n
        assert hasattr(lib, n)


def test_options_default(lib):
    o = dr.dr_options_default()
    assert (o.precision, o.tol, o.max_iter, o.damping, o.dt_safety, o.block, o.placement, o.chunk,
            o.stall_window, o.energy_tol) == (dr.DR_FP64, 1e-8, 2000000, 1e-3, 0.9, 0, dr.DR_PLACE_AUTO,
                                              0, 0, 0.0)


def _packed():
    return I.small_batch(3, 40, 60, 0.01, seed=3).packed()


def _expect_invalid(pk, opt=None, match=""):
    with pytest.raises(dr.DrError) as e:
        dr.dr_batch_create(pk, opt or dr.dr_options_default())
    assert e.value.status == dr.DR_E_INVALID
    assert match in str(e.value), str(e.value)


def test_rejects_bad_networks(lib):
    pk = _packed()
    bad = dict(pk); bad["EA"] = pk["EA"].copy(); bad["EA"][7] = np.nan
    _expect_invalid(bad, match="problem 0 fiber 7")
    bad = dict(pk); bad["EA"] = pk["EA"].copy(); bad["EA"][pk["fiber_offsets"][1] + 2] = 0.0
    _expect_invalid(bad, match="problem 1 fiber 2")
    bad = dict(pk); bad["fiber_nodes"] = pk["fiber_nodes"].copy(); bad["fiber_nodes"][4, 1] = 999
    _expect_invalid(bad, match="out of range")
    bad = dict(pk); bad["fiber_nodes"] = pk["fiber_nodes"].copy()
    bad["fiber_nodes"][5, 1] = bad["fiber_nodes"][5, 0]
    _expect_invalid(bad, match="to itself")
    bad = dict(pk); bad["X"] = pk["X"].copy(); bad["X"][3, 2] = np.inf
    _expect_invalid(bad, match="not finite")
    # a zero-length fiber
    bad = dict(pk); bad["X"] = pk["X"].copy()
    a, b = pk["fiber_nodes"][0]
    bad["X"][b] = bad["X"][a]
    _expect_invalid(bad, match="zero reference length")
    # a free node without fibers
    net = I.Network(np.random.default_rng(0).random((4, 3)), np.array([[0, 1], [1, 2]], np.int32),
                    np.ones(2), np.array([1, 0, 1, 0], np.uint8))
    _expect_invalid(I.Batch([net], np.eye(3)[None]).packed(), match="node 3 is free but has no fiber")
    bad = dict(pk); bad["node_offsets"] = pk["node_offsets"].copy(); bad["node_offsets"][2] = bad["node_offsets"][1]
    _expect_invalid(bad, match="has no nodes")
    # more nodes than one problem may have (the offsets alone are checked first)
    bad = dict(pk); bad["node_offsets"] = pk["node_offsets"].copy(); bad["node_offsets"][1] = 524289
    bad["node_offsets"][2:] = np.maximum(bad["node_offsets"][2:], 524289)
    _expect_invalid(bad, match="at most 524288 per problem")


def test_rejects_bad_options(lib):
    pk = _packed()
    for field, value, msg in [("tol", 0.0, "tol"), ("max_iter", 0, "max_iter"),
                              ("damping", -1.0, "damping"), ("dt_safety", 1.5, "dt_safety"),
                              ("block", 128, "block"), ("placement", 7, "placement"),
                              ("chunk", 3, "chunk"), ("stall_window", -1, "stall_window"),
                              ("energy_tol", -0.5, "energy_tol"), ("energy_tol", float("nan"), "energy_tol"),
                              ("precision", 5, "precision")]:
        o = dr.dr_options_default()
        setattr(o, field, value)
        _expect_invalid(pk, o, msg)
    # LDS placement cannot hold a 7000-node problem
    big = I.Batch([I.draw_network(np.random.default_rng(1), 7000)], np.eye(3)[None]).packed()
    o = dr.dr_options_default(); o.placement = dr.DR_PLACE_LDS
    _expect_invalid(big, o, "DR_PLACE_LDS")


def test_null_arguments(lib):
    import ctypes as C
    o = dr.dr_options_default()
    h = C.c_void_p()
    assert lib.dr_batch_create(None, C.byref(o), None, C.byref(h)) == dr.DR_E_INVALID
    assert "NULL" in dr.dr_last_error()
    assert lib.dr_solve(None, None, None, 1, 0) == dr.DR_E_INVALID
    assert lib.dr_stress(None, None, None, None, None, None, None, None) == dr.DR_E_INVALID
    lib.dr_batch_destroy(None)  # ignored


def test_workspace_bytes_host_only(lib):
    import ctypes as C
    pk = _packed()
    nodes = int(pk["node_offsets"][-1])
    o = dr.dr_options_default()
    n = dr.dr_batch_workspace_bytes(pk, o)
    # every array rounded up to 256 bytes; u (24 B) and the two 32-byte state
    # records per node alone
    assert n % 256 == 0 and n >= nodes * (24 + 32 + 32)
    o2 = dr.dr_options_default(); o2.energy_tol = 0.1
    assert dr.dr_batch_workspace_bytes(pk, o2) - n == (32 * nodes + 255) // 256 * 256  # energy records
    o3 = dr.dr_options_default(); o3.precision = dr.DR_FP32
    assert dr.dr_batch_workspace_bytes(pk, o3) > n  # FP32 copies of the constants
    # the same validation as at create
    bad = dict(pk); bad["EA"] = pk["EA"].copy(); bad["EA"][7] = np.nan
    with pytest.raises(dr.DrError) as e:
        dr.dr_batch_workspace_bytes(bad, o)
    assert e.value.status == dr.DR_E_INVALID and "problem 0 fiber 7" in str(e.value)
    # NULL and unaligned arguments are rejected before any device call
    nets, keep = dr.pack_networks(pk)
    sz = C.c_size_t(7)
    assert lib.dr_batch_workspace_bytes(C.byref(nets), C.byref(o), None) == dr.DR_E_INVALID
    assert lib.dr_batch_workspace_bytes(None, C.byref(o), C.byref(sz)) == dr.DR_E_INVALID and sz.value == 0
    h = C.c_void_p()
    assert lib.dr_batch_create_in(C.byref(nets), C.byref(o), None, None, 1 << 20, C.byref(h)) == dr.DR_E_INVALID
    assert "NULL" in dr.dr_last_error() and h.value is None
    assert lib.dr_batch_create_in(C.byref(nets), C.byref(o), None, C.c_void_p(4104), 1 << 20,
                                  C.byref(h)) == dr.DR_E_INVALID
    assert "aligned" in dr.dr_last_error()
    del keep


def test_pool_arguments_checked_before_device(lib):
    import ctypes as C
    pk = _packed()
    nets, keep = dr.pack_networks(pk)
    o = dr.dr_options_default()
    h = C.c_void_p()
    assert lib.dr_pool_create(C.byref(nets), C.byref(o), None, 0, 4, 100, None) == dr.DR_E_INVALID
    for budget, slots, tick, msg in [(-1, 4, 100, "state_budget_bytes"), (0, 0, 100, "max_slots"),
                                     (0, 4, 0, "tick_passes")]:
        assert lib.dr_pool_create(C.byref(nets), C.byref(o), None, budget, slots, tick,
                                  C.byref(h)) == dr.DR_E_INVALID
        assert msg in dr.dr_last_error() and h.value is None
    F = np.eye(3).ravel()
    n = C.c_int32(5)
    assert lib.dr_pool_submit(None, 0, F.ctypes.data, 1) == dr.DR_E_INVALID
    assert lib.dr_pool_poll(None, 4, None, None, None, None, None, C.byref(n)) == dr.DR_E_INVALID
    assert lib.dr_pool_status(None, None, None, None, None) == dr.DR_E_INVALID
    lib.dr_pool_destroy(None)  # ignored
    del keep


def test_empty_batch_rejected(lib):
    pk = dict(node_offsets=np.zeros(1, np.int64), fiber_offsets=np.zeros(1, np.int64), X=np.zeros((0, 3)),
              fiber_nodes=np.zeros((0, 2), np.int32), EA=np.zeros(0), fixed=np.zeros(0, np.uint8), band=0.02)
    with pytest.raises(dr.DrError) as e:
        dr.dr_batch_workspace_bytes(pk, dr.dr_options_default())
    assert e.value.status == dr.DR_E_INVALID and "n_problems" in str(e.value)


def test_band_rule_when_fixed_is_null(lib):
    """fixed = NULL: a node is prescribed iff it lies within `band` of a face
    (inclusive).  Node 2 sits in the middle without a fiber: free (and
    rejected) at band 0.02, prescribed (and accepted) at band 0.5; nodes 0
    and 1 lie 0.01 from a face."""
    X = np.array([[0.01, 0.5, 0.5], [0.99, 0.5, 0.5], [0.5, 0.5, 0.5]])
    base = dict(node_offsets=np.array([0, 3], np.int64), fiber_offsets=np.array([0, 1], np.int64), X=X,
                fiber_nodes=np.array([[0, 1]], np.int32), EA=np.ones(1), fixed=None)
    o = dr.dr_options_default()
    with pytest.raises(dr.DrError) as e:
        dr.dr_batch_workspace_bytes(dict(base, band=0.02), o)
    assert e.value.status == dr.DR_E_INVALID and "node 2 is free but has no fiber" in str(e.value)
    n_band = dr.dr_batch_workspace_bytes(dict(base, band=0.5), o)
    n_mask = dr.dr_batch_workspace_bytes(dict(base, fixed=np.ones(3, np.uint8)), o)
    assert n_band == n_mask > 0
    # exactly at the band distance counts as prescribed
    with pytest.raises(dr.DrError):
        dr.dr_batch_workspace_bytes(dict(base, band=0.4999), o)
    assert dr.dr_batch_workspace_bytes(dict(base, band=0.5), o) > 0
    for bad in (-0.1, float("nan"), float("inf")):
        with pytest.raises(dr.DrError) as e:
            dr.dr_batch_workspace_bytes(dict(base, band=bad), o)
        assert e.value.status == dr.DR_E_INVALID and "band" in str(e.value)
    # the band rule on a workload network gives the generator's mask
    pk = I.small_batch(2, 300, 400, 0.01, seed=5).packed()
    assert dr.dr_batch_workspace_bytes(dict(pk, fixed=None, band=I.BAND), o) == \
        dr.dr_batch_workspace_bytes(pk, o)


def test_state_bytes_per_node(lib):
    """Two state records and one velocity record per node: 2 x 24 + 24 in
    FP64, 2 x 32 + 16 in FP32."""
    assert dr.state_bytes_per_node(dr.DR_FP64) == 72
    assert dr.state_bytes_per_node(dr.DR_FP32) == 80
    with pytest.raises(dr.DrError):
        dr.state_bytes_per_node(7)


def test_global_256_threads_runs_chunks_of_one(lib):
    """Global placement with 256 threads has only a chunk-1 build: asking for
    chunks of 2 or 4 there is an error, not a silent substitution."""
    pk = _packed()
    for ch in (2, 4):
        o = dr.dr_options_default()
        o.placement, o.block, o.chunk = dr.DR_PLACE_GLOBAL, 256, ch
        with pytest.raises(dr.DrError) as e:
            dr.dr_batch_workspace_bytes(pk, o)
        assert e.value.status == dr.DR_E_INVALID and "chunks of 1" in str(e.value)
    o = dr.dr_options_default()
    o.placement, o.block, o.chunk = dr.DR_PLACE_GLOBAL, 256, 1
    assert dr.dr_batch_workspace_bytes(pk, o) > 0


def test_rejects_bad_step_rule_options(lib):
    """The per-pass step (dt_rule 1) is FP64 only, without the energy check
    and without the tail hand-off; its group form takes 2..16 workgroups."""
    pk = _packed()
    cases = [(dict(dt_rule=2), "dt_rule"), (dict(dt_rule=1, precision=dr.DR_FP32), "FP64"),
             (dict(dt_rule=1, energy_tol=1e-3), "energy"), (dict(dt_rule=1, tail_at=4), "hand-off"),
             (dict(dt_rule=1, tail_group=1), "tail_group"), (dict(dt_rule=1, tail_group=17), "tail_group")]
    for kw, msg in cases:
        o = dr.dr_options_default()
        for k, v in kw.items():
            setattr(o, k, v)
        _expect_invalid(pk, o, msg)


def test_tiles_only_above_the_lds_limit(lib):
    """A problem of more than 6720 nodes (too large for the LDS variant) is
    packed with tiles: a 2-byte neighbour slot per incidence entry (at least
    two per fiber) plus its tiles' halo lists, which the workspace accounts
    for; a batch whose problems all fit in LDS carries none."""
    rng = np.random.default_rng(5)

    def bytes_for(n):
        net = I.draw_network(rng, n)
        pk = I.Batch([net], np.eye(3)[None]).packed()
        return dr.dr_batch_workspace_bytes(pk, dr.dr_options_default()), net.n_fibers
    small, m_small = bytes_for(6720)
    big, m_big = bytes_for(6721)
    # the two networks differ by a few fibers (per fiber: two 20-byte
    # incidence entries, two degrees' worth of rounding); 256-byte rounding
    # of every array
    slack = 64 * abs(m_big - m_small) + 64 * 256
    assert big - small >= 2 * 2 * m_big - slack
