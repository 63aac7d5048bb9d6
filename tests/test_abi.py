"""The C-ABI library loads, exports every entry point declared in include/dgmg.h,
and its host-side setup validates arguments and matches the oracle's geometry.
No device work is started here."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth
from paper_1603_02524_amd import dgmg as D

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dgmg.h")


def _header_symbols():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(dgmg_\w+)\s*\(", txt, re.M)))


def test_library_exports_every_declared_symbol():
    lib = D.load_library()
    syms = _header_symbols()
    assert len(syms) >= 34
    for s in syms:
        assert hasattr(lib, s), s
    assert sorted(n for n, _, _ in D.SIGNATURES) == syms


def test_struct_layouts_match_header():
    # dgmg_stats holds 256 history entries; sizes follow the C declaration order
    assert ctypes.sizeof(D.DgmgStats) == 4 + 4 + 8 * 3 + 8 * 256 + 8 + 4 + 4  # r_true, replacements, tail padding
    # int dim; int n_elem[3]; const double* dx[3] (8-aligned at 16); int periodic[3]; tail pad
    assert ctypes.sizeof(D.DgmgGrid) == 56
    assert ctypes.sizeof(D.DgmgOpts) == 4 + 4 + 24 + 8 + 4 * 10  # ... order, disc


def test_defaults():
    lib = D.load_library()
    o = D.DgmgOpts()
    assert lib.dgmg_opts_default(ctypes.byref(o)) == 0
    assert o.P == 4 and o.mu_star == 1.0 and o.ns_pre == 1 and o.ns_post == 1 and o.overlap == -1


@pytest.mark.parametrize("bad", [
    dict(P=33), dict(P=0), dict(P=20), dict(mu_star=0.0), dict(mu_star=-1.0), dict(smoother="XX"),
])
def test_setup_rejects_bad_options(bad):
    g = synth.uniform_grid(3, 2, 1.0, False)
    m = synth.Method(P=4)
    for k, v in bad.items():
        setattr(m, k, v)
    if bad.get("smoother") == "XX":
        with pytest.raises(KeyError):
            D.setup_handle(g, m)
        return
    with pytest.raises(D.DgmgError) as ei:
        D.setup_handle(g, m)
    assert ei.value.code < 0


def test_setup_rejects_bad_grid():
    m = synth.Method(P=4)
    g = synth.Grid(3, (np.array([0.5, -0.5]), np.ones(2), np.ones(2)), (False,) * 3)
    with pytest.raises(D.DgmgError):
        D.setup_handle(g, m)
    g = synth.Grid(3, (np.array([0.5, np.nan]), np.ones(2), np.ones(2)), (False,) * 3)
    with pytest.raises(D.DgmgError):
        D.setup_handle(g, m)
    g = synth.uniform_grid(3, 2, 1.0, True)          # periodic needs >= 3 elements
    with pytest.raises(D.DgmgError):
        D.setup_handle(g, m)
    g = synth.uniform_grid(2, 3, 1.0, False)
    with pytest.raises(D.DgmgError):
        D.setup_handle(g, synth.Method(P=4, flux="ldg", beta=(2.0, 0.0)))


def test_level_series_and_geometry_match_oracle():
    from oracle import multigrid as mg
    from oracle import operator as op
    from oracle.schwarz import overlap_for
    lib = D.load_library()
    rng = np.random.default_rng(0)
    g = synth.Grid(3, tuple(rng.uniform(0.2, 1.0, 3) for _ in range(3)), (False,) * 3)
    for P in (1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 13, 16, 17):
        for ov in ("level", "level_floor", "zero"):
            m = synth.Method(P=P, smoother="FA", overlap=ov)
            h, keep = D.setup_handle(g, m)
            try:
                orders = mg.level_orders(P)
                assert lib.dgmg_num_levels(h) == len(orders)
                for l, Pl in enumerate(orders):
                    Pc, no, nd = ctypes.c_int(), ctypes.c_int(), ctypes.c_int64()
                    assert lib.dgmg_level_info(h, l, ctypes.byref(Pc), ctypes.byref(no), ctypes.byref(nd)) == 0
                    assert Pc.value == Pl and nd.value == g.n_elem * (Pl + 1) ** 3
                    assert no.value == (overlap_for(Pl, ov) if l > 0 else 0)
                    x = np.zeros(3 * (Pl + 1))
                    assert lib.dgmg_node_coords(h, l, 0, x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) == 0
                    assert np.allclose(x, op.node_coords_1d(np.asarray(g.dx[0]), Pl), atol=1e-15)
                # device entry points refuse to run before a workspace is bound
                assert lib.dgmg_apply(h, 0, ctypes.c_void_p(8), ctypes.c_void_p(16), 0) == D.DgmgError(-3, "").code
                assert b"workspace" in lib.dgmg_last_error(h)
            finally:
                lib.dgmg_destroy(h)


def test_kernel_timing_rejects_a_negative_stride():
    """dgmg_kernel_timing(h, k): k >= 1 times every k-th top-level patch-solve
    launch, 0 stops; a negative stride is refused before any HIP call."""
    lib = D.load_library()
    g = synth.uniform_grid(3, 2, 1.0, False)
    h, keep = D.setup_handle(g, synth.Method(P=2, smoother="FA"))
    try:
        assert lib.dgmg_kernel_timing(h, -1) == -1  # DGMG_EINVAL
        assert b"negative stride" in lib.dgmg_last_error(h)
    finally:
        lib.dgmg_destroy(h)


def test_batch_layout_host_side():
    """Batch setup (host only): member workspaces are disjoint, aligned and inside
    the batch workspace; unknown offsets follow the member sizes."""
    lib = D.load_library()
    rng = np.random.default_rng(1)
    probs = []
    for P in (4, 6, 8, 2, 12, 3):
        n = tuple(int(v) for v in rng.integers(1, 4, size=3))
        probs.append((synth.Grid(3, tuple(rng.uniform(0.5, 1.5, n[d]) for d in range(3)), (False,) * 3),
                      synth.Method(P=P, smoother="FA")))
    k = len(probs)
    grids = (D.DgmgGrid * k)()
    opts = (D.DgmgOpts * k)()
    keep = []
    for i, (g, m) in enumerate(probs):
        gg, oo, kk = D.make_structs(g, m)
        grids[i], opts[i] = gg, oo
        keep.append(kk)
    b = ctypes.c_void_p()
    assert lib.dgmg_batch_setup(k, grids, opts, ctypes.byref(b)) == 0
    try:
        total = ctypes.c_size_t()
        assert lib.dgmg_batch_workspace_bytes(b, ctypes.byref(total)) == 0
        sizes = []
        for i in range(k):
            h = ctypes.c_void_p()
            assert lib.dgmg_batch_handle(b, i, ctypes.byref(h)) == 0
            nb = ctypes.c_size_t()
            assert lib.dgmg_workspace_bytes(h, ctypes.byref(nb)) == 0
            sizes.append(nb.value)
        assert total.value >= sum(sizes)
        off = (ctypes.c_int64 * (k + 1))()
        assert lib.dgmg_batch_offsets(b, off) == 0
        for i, (g, m) in enumerate(probs):
            assert off[i + 1] - off[i] == g.n_dof(m.P)
    finally:
        lib.dgmg_batch_destroy(b)


@pytest.mark.parametrize("name", ["c1", "c5", "periodic"])
def test_face_features_match_oracle(name):
    """Per-face MLP features computed by the library's host setup equal the oracle's."""
    from oracle import learned
    from paper_1603_02524_amd import dgmg
    if name == "c1":
        w = synth.with_method(synth.c1_poisson2d_p4(), smoother="FA")
    elif name == "c5":
        w = synth.c5_poisson3d_p32(n=3)
    else:
        w = synth.paper_periodic_2d(8, n=4, ar=4, smoother="FA")
    X = dgmg.face_features(w.grid, w.method)
    ref = learned.face_features(w.grid, w.method)
    assert X.shape == ref.shape
    assert np.allclose(X, ref, rtol=0, atol=2e-7)


def _batch(lib, probs):
    k = len(probs)
    grids = (D.DgmgGrid * k)()
    opts = (D.DgmgOpts * k)()
    keep = []
    for i, (g, m) in enumerate(probs):
        gg, oo, kk = D.make_structs(g, m)
        grids[i], opts[i] = gg, oo
        keep.append(kk)
    b = ctypes.c_void_p()
    assert lib.dgmg_batch_setup(k, grids, opts, ctypes.byref(b)) == 0
    return b, keep


def _plan(lib, b):
    p, kk, g = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    assert lib.dgmg_batch_plan_info(b, ctypes.byref(p), ctypes.byref(kk), ctypes.byref(g)) == 0
    return p.value, kk.value, g.value


def test_batch_plan_host_side():
    """The batched execution plan (host only, before any device memory): grids of
    one precision and smoothing schedule merge their kernel steps into shared
    launches, so the launch count per iteration grows with the number of distinct
    (order, tile) shapes, not with the number of grids; a multiplicative grid in
    the batch turns the plan off (each grid then issues its own chain)."""
    lib = D.load_library()
    rng = np.random.default_rng(2)

    def grid(n):
        return synth.Grid(3, tuple(rng.uniform(0.5, 1.5, n) for _ in range(3)), (False,) * 3)

    one = [(grid(2), synth.Method(P=8, smoother="FA", precision="mixed"))]
    many = one + [(grid(int(rng.integers(1, 4))), synth.Method(P=8, smoother="FA", precision="mixed"))
                  for _ in range(15)]
    b1, k1 = _batch(lib, one)
    b16, k16 = _batch(lib, many)
    try:
        p1, n1, g1 = _plan(lib, b1)
        p16, n16, g16 = _plan(lib, b16)
        assert p1 == 1 and p16 == 1
        assert n16 == n1                    # same orders and tiles: the same launches, 16 grids each
        assert g16 == 16 * g1               # per-grid operations scale with the grids
    finally:
        lib.dgmg_batch_destroy(b1)
        lib.dgmg_batch_destroy(b16)
    mixed_kinds = [(grid(2), synth.Method(P=4, smoother="FA")), (grid(2), synth.Method(P=4, smoother="FM"))]
    b, k = _batch(lib, mixed_kinds)
    try:
        assert _plan(lib, b)[0] == 0
    finally:
        lib.dgmg_batch_destroy(b)


@pytest.mark.parametrize("dim,n,periodic,P", [(2, (5, 3), False, 4), (2, (4, 3), True, 32), (3, (3, 2, 3), (True, False, False), 6),
                                              (3, (2, 2, 2), False, 16), (3, (3, 4, 3), True, 2)])
def test_continuous_setup_matches_oracle_lattice(dim, n, periodic, P):
    """Continuous handles (host only): level sizes, overlaps and lattice node
    coordinates equal the oracle's."""
    from oracle import se
    lib = D.load_library()
    rng = np.random.default_rng(3)
    per = periodic if isinstance(periodic, tuple) else (periodic,) * dim
    g = synth.Grid(dim, tuple(rng.uniform(0.4, 1.6, n[d]) for d in range(dim)), per)
    m = synth.Method(P=P, smoother="EA", disc="se")
    h, keep = D.setup_handle(g, m)
    try:
        from oracle import multigrid as mg
        orders = mg.level_orders(P)
        assert lib.dgmg_num_levels(h) == len(orders)
        for l, Pl in enumerate(orders):
            Pc, no, nd = ctypes.c_int(), ctypes.c_int(), ctypes.c_int64()
            assert lib.dgmg_level_info(h, l, ctypes.byref(Pc), ctypes.byref(no), ctypes.byref(nd)) == 0
            assert Pc.value == Pl and nd.value == se.n_dof(g, Pl) == g.n_lattice(Pl)
            if l > 0:
                assert no.value == se.se_overlap(Pl, "level")
            for d in range(dim):
                ref = se.node_coords_1d(g.dx[d], Pl, per[d])
                x = np.zeros(len(ref))
                assert lib.dgmg_node_coords(h, l, d, x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) == 0
                assert np.allclose(x, ref, rtol=0, atol=1e-14)
    finally:
        lib.dgmg_destroy(h)


def test_continuous_unsupported_configurations_are_rejected():
    g = synth.uniform_grid(3, 2, 1.0, False)
    for m in (synth.Method(P=4, smoother="FA", disc="se"), synth.Method(P=32, smoother="EA", disc="se"),
              synth.Method(P=4, smoother="EA", overlap="zero", disc="se"),
              synth.Method(P=4, smoother="EM", disc="se")):
        with pytest.raises(D.DgmgError):
            D.setup_handle(g, m)
    # a Dirichlet direction of one element has no coarse unknowns
    g1 = synth.Grid(3, (np.ones(1), np.ones(2), np.ones(2)), (False,) * 3)
    with pytest.raises(D.DgmgError):
        D.setup_handle(g1, synth.Method(P=4, smoother="EA", disc="se"))
    # batches take DG grids only
    lib = D.load_library()
    probs = [(g, synth.Method(P=4, smoother="EA", disc="se"))]
    grids = (D.DgmgGrid * 1)()
    opts = (D.DgmgOpts * 1)()
    gg, oo, kk = D.make_structs(*probs[0])
    grids[0], opts[0] = gg, oo
    b = ctypes.c_void_p()
    assert lib.dgmg_batch_setup(1, grids, opts, ctypes.byref(b)) == D.DgmgError(-4, "").code
