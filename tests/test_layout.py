"""Host SlimSell layout: the invariants of Sections II-D and III-B.

L1 rows hold exactly their neighbour sets (relabelled), L2 the cell counts of
Table "sizes", L3 the padding bound of the work analysis (Section III-A,
"Work Complexity"), L4 sigma below C gives no padding reduction, L5 rows are
sorted inside each sigma window, plus argument errors.  No GPU is used.
"""
import re

import numpy as np
import pytest

import graphgen
import oracle
import paper_2010_09913_amd as ss
from paper_2010_09913_amd import _native

C = 64


def _rows_of(L):
    """Set of (row, col) pairs stored in the layout, ignoring padding."""
    out = []
    for i in range(L.n_chunks):
        ncol = L.cl[i]
        blk = L.col[L.cs[i]:L.cs[i + 1]].reshape(ncol, C) if ncol else np.zeros((0, C), np.int32)
        jj, lane = np.nonzero(blk >= 0)
        out.append(np.stack([i * C + lane, blk[jj, lane]], 1))
    return np.concatenate(out) if out else np.zeros((0, 2), np.int64)


@pytest.mark.parametrize("kind,sigma", [("rmat", 0), ("rmat", 1), ("rmat", 64), ("rmat", 1024),
                                        ("er", 0), ("er", 128), ("grid", 0)])
def test_layout_invariants(kind, sigma):
    if kind == "rmat":
        e = graphgen.rmat(11, 16, seed=1)
    elif kind == "er":
        e = graphgen.er(3000, 20000, seed=2)
    else:
        e = graphgen.grid(45, 37, 0.05, seed=5)
    L = ss.layout_build(e.src, e.dst, e.n, sigma=sigma)
    g = oracle.csr_from_edgelist(e)
    n_pad = (e.n + C - 1) // C * C
    assert L.n == e.n and L.n_pad == n_pad and L.n_chunks == n_pad // C
    # relabelling is a bijection and v is its inverse (1-based)
    assert sorted(L.perm.tolist()) == sorted(set(L.perm.tolist()))
    np.testing.assert_array_equal(L.v[L.perm], np.arange(e.n) + 1)
    assert np.all(L.v[np.setdiff1d(np.arange(n_pad), L.perm)] == 0)
    # L1: non-marker cells of each row = its neighbour set through perm
    stored = _rows_of(L)
    rows = np.repeat(np.arange(g.n), np.diff(g.rowptr))
    want = np.stack([L.perm[rows], L.perm[g.adj]], 1)
    key = lambda a: np.sort(a[:, 0].astype(np.int64) * n_pad + a[:, 1])
    np.testing.assert_array_equal(key(stored), key(want))
    assert np.all((L.col >= -1) & (L.col < n_pad))
    # each row lists its neighbours by strictly decreasing original ID (the
    # sel-max scan stops at the first frontier neighbour)
    for i in range(0, L.n_chunks, max(1, L.n_chunks // 40)):
        blk = L.col[L.cs[i]:L.cs[i + 1]].reshape(-1, C)
        for lane in range(C):
            nb = blk[:, lane]
            ids = L.v[nb[nb >= 0]] - 1
            assert np.all(np.diff(ids) < 0)
    # L2: E + P cells, cs is the prefix of C * cl
    assert L.entries == g.entries
    assert L.cells == C * int(L.cl.sum()) == L.cs[-1]
    np.testing.assert_array_equal(np.diff(L.cs), C * L.cl.astype(np.int64))
    np.testing.assert_array_equal(L.degree[L.perm], g.degree)
    for i in range(L.n_chunks):
        assert L.cl[i] == L.degree[i * C:(i + 1) * C].max()
    # L5: rows sorted by decreasing degree inside every window, stable on the ID
    win = n_pad if sigma in (0, e.n) else sigma
    if win > 1:
        deg_rows = L.degree
        for w0 in range(0, n_pad, win):
            seg = deg_rows[w0:w0 + win]
            assert np.all(seg[:-1] >= seg[1:])
            ids = L.v[w0:w0 + win] - 1
            real = ids >= 0
            # the window holds exactly the IDs of that window
            assert set(ids[real].tolist()) == set(range(w0, min(w0 + win, e.n)))
            for dval in np.unique(seg[real]):
                same = ids[real][seg[real] == dval]
                assert np.all(np.diff(same) > 0)
    else:
        np.testing.assert_array_equal(L.v[:e.n], np.arange(e.n) + 1)


def test_padding_bound_at_full_sort():
    # L3: with full sorting the padding is at most C times the maximum degree
    for e in (graphgen.rmat(12, 16, seed=1), graphgen.er(5000, 80000, seed=2)):
        L = ss.layout_build(e.src, e.dst, e.n, sigma=0)
        assert L.padding <= C * L.max_cl
        assert L.max_cl == L.degree.max()


def test_sigma_below_chunk_height_gives_no_padding_reduction():
    # L4: sigma < C only reorders rows inside chunks; our sigma=1 is that case and
    # its padding equals that of the unsorted degree sequence chunked by 64
    e = graphgen.rmat(11, 16, seed=4)
    L1 = ss.layout_build(e.src, e.dst, e.n, sigma=1)
    g = oracle.csr_from_edgelist(e)
    deg = np.zeros(L1.n_pad, np.int64)
    deg[:e.n] = g.degree
    pad = int((deg.reshape(-1, C).max(1) * C - deg.reshape(-1, C).sum(1)).sum())
    assert L1.padding == pad
    Ln = ss.layout_build(e.src, e.dst, e.n, sigma=0)
    assert Ln.padding < L1.padding


def test_storage_formulas_of_table_sizes():
    # Table "sizes": SlimSell 2m + 2n/C + P cells vs Sell-C-sigma 4m + 2n/C + P,
    # CSR 4m + n and AL 2m + n (m undirected edges, E = 2m directed cells)
    e = graphgen.rmat(13, 16, seed=1)
    L = ss.layout_build(e.src, e.dst, e.n, sigma=0)
    E = L.entries
    slim = L.cells + 2 * L.n_chunks
    sell = 2 * E + 2 * L.n_chunks + 2 * L.padding
    al = E + L.n
    assert slim == E + 2 * L.n_chunks + L.padding
    assert slim < sell
    # AL inequality of Section III-B: SlimSell is smaller iff P < n (1 - 2/C)
    assert (slim < al) == (L.padding < L.n_pad * (1 - 2 / C))


def test_isolated_vertices_and_phantom_rows():
    L = ss.layout_build([0, 1], [1, 2], 70, sigma=0)
    assert L.n_pad == 128 and L.n_chunks == 2
    assert L.entries == 4 and L.max_cl == 2
    assert L.cl[1] == 0
    assert L.v[70:].tolist() == [0] * 58


@pytest.mark.parametrize("args,msg", [
    (dict(n=0), "n must be"),
    (dict(C=32), "C must be 64"),
    (dict(sigma=96), "sigma"),    # not a multiple of 64
    (dict(sigma=256), "sigma"),   # > padded 128
    (dict(src=[0, 500]), "out of range"),
])
def test_layout_argument_errors(args, msg):
    kw = dict(src=[0, 1], dst=[1, 2], n=100, sigma=0, C=64)
    kw.update(args)
    with pytest.raises(ss.SlimSellError) as ei:
        ss.layout_build(kw["src"], kw["dst"][:len(kw["src"])], kw["n"], sigma=kw["sigma"],
                        C=kw["C"])
    assert ei.value.code == _native.SS_EINVAL
    assert msg in str(ei.value)


def test_library_exports_every_declared_symbol():
    import ctypes
    import os
    hdr = open(os.path.join(os.path.dirname(__file__), "..", "include", "slimsell.h")).read()
    declared = set(re.findall(r"^\s*(?:const\s+)?[\w\s\*]*?\b(slimsell_\w+)\s*\(", hdr, re.M))
    assert declared == set(_native.EXPORTS)
    lib = ctypes.CDLL(_native.LIB_PATH)
    for name in declared:
        assert hasattr(lib, name), name
    assert "gfx950" in ss.version()


def test_build_without_device_reports_unsupported_or_builds():
    # On a machine without a HIP device the upload step must fail cleanly.
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    with pytest.raises(ss.SlimSellError) as ei:
        ss.Graph([0, 1], [1, 2], 3)
    assert ei.value.code in (_native.SS_EUNSUP, _native.SS_EHIP)


def test_storage_against_table_sizes():
    """Table "sizes": SlimSell needs about half of Sell-C-sigma (which stores val
    as well as col) and less than CSR, and it is smaller than AL exactly when
    the padding stays below n(1 - 2/C) (the inequality of Section III-B)."""
    import paper_2010_09913_amd as ss
    for e in (graphgen.rmat(14, 16, seed=1), graphgen.er(1 << 14, 40 << 14, seed=2)):
        for sigma in (0, 1024, 1):
            L = ss.layout_build(e.src, e.dst, e.n, sigma=sigma, arrays=False)
            E, P, nc = L.entries, L.cells - L.entries, L.n_chunks
            assert nc * 64 == e.n
            slim, sell, csr, al = E + P + 2 * nc, 2 * (E + P) + 2 * nc, 2 * E + e.n, E + e.n
            assert 0.5 < slim / sell < 0.51
            if sigma == 0:
                assert slim < csr
            assert (slim < al) == (P < e.n * (1 - 2 / 64))
