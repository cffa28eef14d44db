"""Host-side checks of the SELL-C-sigma storage (chunk height C, sorting
window sigma; section "Related Work" of the paper for the format, section
"Testbed and Implementation" for C = 1 as CRS): the layout the library
computes, an independent NumPy product through that layout, the import's
argument validation before any device call, and the irregular-matrix input
generator."""
import ctypes
import os

import numpy as np
import pytest

from paper_1410_5242_amd import inputs


@pytest.fixture(scope="module")
def kpm():
    from paper_1410_5242_amd import kpm as k
    if not os.path.exists(k.LIB_PATH):
        pytest.skip("libkpm.so not built (run __graft_entry__.build())")
    k.lib()
    return k


def _lengths(rowptr):
    return np.diff(np.asarray(rowptr, dtype=np.int64))


@pytest.mark.parametrize("C,sigma", [(1, 1), (2, 4), (4, 1), (8, 64), (32, 32), (32, 256), (64, 1 << 20)])
def test_layout_sorts_windows_and_sizes_chunks(kpm, C, sigma):
    rowptr, _, _ = inputs.random_hermitian_csr(1000, seed=7)
    lens = _lengths(rowptr)
    perm, width, start = kpm.sell_layout(rowptr, C, sigma)
    N = lens.size
    assert sorted(perm.tolist()) == list(range(N))          # every row exactly once
    for w0 in range(0, N, sigma):
        w1 = min(N, w0 + sigma)
        win = perm[w0:w1]
        assert set(win.tolist()) == set(range(w0, w1))         # rows stay in their window
        l = lens[win]
        assert np.all(l[:-1] >= l[1:])                          # decreasing length
        for a, b in zip(win[:-1], win[1:]):                     # stable among equal lengths
            if lens[a] == lens[b]:
                assert a < b
    nch = (N + C - 1) // C
    assert width.size == nch and start.size == nch + 1 and start[0] == 0
    for c in range(nch):
        assert width[c] == lens[perm[c * C:(c + 1) * C]].max()
        assert start[c + 1] - start[c] == C * width[c]


def test_layout_with_c1_and_no_sorting_is_crs(kpm):
    rowptr, _, _ = inputs.random_hermitian_csr(777, seed=2)
    perm, width, start = kpm.sell_layout(rowptr, 1, 1)
    assert np.array_equal(perm, np.arange(777))
    assert np.array_equal(start, rowptr)
    assert np.array_equal(width, _lengths(rowptr))


def test_sorting_cuts_padding_on_an_irregular_matrix(kpm):
    rowptr, _, _ = inputs.random_hermitian_csr(20000, seed=5)
    nnz = int(rowptr[-1])
    _, _, s_unsorted = kpm.sell_layout(rowptr, 32, 1)
    _, _, s_sorted = kpm.sell_layout(rowptr, 32, 256)
    _, _, s_global = kpm.sell_layout(rowptr, 32, 1 << 16)
    assert s_unsorted[-1] > 2.0 * nnz                  # long tail: unsorted chunks pad a lot
    assert s_global[-1] <= s_sorted[-1] < s_unsorted[-1]
    assert s_global[-1] < 1.05 * nnz + 32 * 256


@pytest.mark.parametrize("C,sigma", [(1, 1), (4, 16), (32, 256)])
def test_product_through_the_layout_equals_crs(kpm, C, sigma):
    # y = H x computed from the SELL arrays assembled here from the layout
    # (entry j of position p at start[p/C] + j C + p mod C; padding: column N,
    # value 0) against the CRS product
    N = 500
    rowptr, col, val = inputs.random_hermitian_csr(N, seed=11)
    perm, width, start = kpm.sell_layout(rowptr, C, sigma)
    scol = np.full(start[-1], N, dtype=np.int64)
    sval = np.zeros(start[-1], dtype=np.complex128)
    for p in range(N):
        r = perm[p]
        e0 = start[p // C] + p % C
        k = np.arange(rowptr[r], rowptr[r + 1])
        scol[e0 + C * np.arange(k.size)] = col[k]
        sval[e0 + C * np.arange(k.size)] = val[k]
    rng = np.random.default_rng(0)
    x = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    xp = np.concatenate([x, [0.0]])
    y = np.zeros(N, dtype=np.complex128)
    for p in range(N):
        e = start[p // C] + p % C + C * np.arange(width[p // C])
        y[perm[p]] = np.sum(sval[e] * xp[scol[e]])
    ref = np.array([np.sum(val[rowptr[i]:rowptr[i + 1]] * x[col[rowptr[i]:rowptr[i + 1]]]) for i in range(N)])
    assert np.allclose(y, ref, rtol=0, atol=1e-12)


def test_layout_rejects_bad_arguments(kpm):
    rp = np.array([0, 2, 3, 3], dtype=np.int64)
    for C, sigma in ((3, 1), (0, 1), (128, 128), (8, 12), (8, 0)):
        with pytest.raises(kpm.KPMError):
            kpm.sell_layout(rp, C, sigma)
    with pytest.raises(kpm.KPMError, match="decreases"):
        kpm.sell_layout(np.array([0, 2, 1], dtype=np.int64), 1, 1)
    with pytest.raises(kpm.KPMError, match="rowptr"):
        kpm.sell_layout(np.array([1, 2], dtype=np.int64), 1, 1)


def test_import_validates_before_any_device_call(kpm):
    L = kpm.lib()
    out = ctypes.c_void_p(1)
    assert L.kpm_import_csr(None, None, ctypes.byref(out)) == kpm.KPM_EINVAL
    assert out.value is None
    rowptr = np.array([0, 2, 3], dtype=np.int64)
    col = np.array([0, 1, 1], dtype=np.int32)
    val = np.array([1.0, 0.0, 0.5, 0.5, 2.0, 0.0])

    def desc(**kw):
        d = kpm.CsrDesc()
        d.N, d.rowptr, d.col, d.val = 2, rowptr.ctypes.data, col.ctypes.data, val.ctypes.data
        d.dtype, d.margin = 0, 1.01
        for k, v in kw.items():
            setattr(d, k, v)
        return d

    cases = [(dict(dtype=7), b"dtype"), (dict(margin=0.5), b"margin"), (dict(sell_C=3), b"power of two"),
             (dict(sell_C=8, sell_sigma=12), b"sigma"), (dict(N=0), b"N must be"),
             (dict(col=None), b"col or val"), (dict(fixed_scale=1, a=-1.0), b"fixed scale")]
    for kw, msg in cases:
        d = desc(**kw)
        assert L.kpm_import_csr(ctypes.byref(d), None, ctypes.byref(out)) == kpm.KPM_EINVAL, kw
        assert msg in L.kpm_last_error(), (kw, L.kpm_last_error())
    bad_col = np.array([0, 2, 1], dtype=np.int32)
    d = desc(col=bad_col.ctypes.data)
    assert L.kpm_import_csr(ctypes.byref(d), None, ctypes.byref(out)) == kpm.KPM_EINVAL
    assert b"column out of range" in L.kpm_last_error()
    bad_val = val.copy()
    bad_val[3] = np.nan
    d = desc(val=bad_val.ctypes.data)
    assert L.kpm_import_csr(ctypes.byref(d), None, ctypes.byref(out)) == kpm.KPM_EINVAL
    assert b"non-finite" in L.kpm_last_error()


def test_irregular_generator_is_hermitian_seeded_and_irregular():
    N = 3000
    rowptr, col, val = inputs.random_hermitian_csr(N, seed=4)
    import scipy.sparse as sp
    A = sp.csr_matrix((val, col, rowptr), shape=(N, N))
    assert abs(A - A.getH()).max() == 0.0
    lens = _lengths(rowptr)
    empty = lens == 0
    assert 0.005 < empty.mean() < 0.05
    assert A[empty].nnz == 0 and A[:, empty].nnz == 0
    assert 9.0 < lens[~empty].mean() < 15.0
    assert lens.max() > 5 * np.median(lens[~empty])      # a long tail of row lengths
    r2, c2, v2 = inputs.random_hermitian_csr(N, seed=4)
    assert np.array_equal(r2, rowptr) and np.array_equal(c2, col) and np.array_equal(v2, val)
    r3, _, _ = inputs.random_hermitian_csr(N, seed=5)
    assert not np.array_equal(r3, rowptr)


def test_lattice_desc_sell_fields_are_validated_before_any_device_call(kpm):
    L = kpm.lib()
    out = ctypes.c_void_p(1)
    d = kpm.LatticeDesc()
    d.L[0] = d.L[1] = d.L[2] = 4
    d.periodic[0] = d.periodic[1] = d.periodic[2] = 1
    d.t, d.margin = 1.0, 1.01
    for C, sigma, msg in ((3, 0, b"sell_C"), (128, 0, b"sell_C"), (-1, 0, b"sell_C"), (8, 12, b"sell_sigma"),
                          (8, -4, b"sell_sigma")):
        d.sell_C, d.sell_sigma = C, sigma
        assert L.kpm_build_hamiltonian(ctypes.byref(d), None, ctypes.byref(out)) == kpm.KPM_EINVAL, (C, sigma)
        assert msg in L.kpm_last_error()
        assert out.value is None


def test_layout_properties_on_random_patterns(kpm):
    # random row-length patterns (empty rows, long rows, N not a multiple of
    # C or sigma) under every chunk height and several sorting windows
    hyp = pytest.importorskip("hypothesis")
    st = hyp.strategies

    @hyp.settings(max_examples=60, deadline=None, derandomize=True)
    @hyp.given(lens=st.lists(st.integers(0, 40), min_size=1, max_size=300),
               logc=st.integers(0, 6), mult=st.sampled_from([0, 1, 2, 5, 1000]))
    def check(lens, logc, mult):
        C = 1 << logc
        sigma = 1 if mult == 0 else C * mult
        lens = np.asarray(lens, dtype=np.int64)
        rowptr = np.concatenate([[0], np.cumsum(lens)])
        perm, width, start = kpm.sell_layout(rowptr, C, sigma)
        N = lens.size
        assert sorted(perm.tolist()) == list(range(N))
        nch = (N + C - 1) // C
        assert width.size == nch and start[0] == 0 and start.size == nch + 1
        for c in range(nch):
            assert width[c] == lens[perm[c * C:(c + 1) * C]].max()
            assert start[c + 1] - start[c] == C * width[c]
        w = 1 if sigma == 1 else sigma
        for w0 in range(0, N, w):
            win = perm[w0:w0 + w]
            assert set(win.tolist()) == set(range(w0, min(N, w0 + w)))
            if sigma > 1:
                assert np.all(lens[win][:-1] >= lens[win][1:])
        # stored entries never below the nonzeros; sorting never pads more
        # than leaving the rows in order
        assert start[-1] >= lens.sum()
        if sigma > 1:
            _, _, s1 = kpm.sell_layout(rowptr, C, 1)
            assert start[-1] <= s1[-1]

    check()
