"""Wavenumber sweeps through one handle (cm_create with n_k wavenumbers,
cm_apply with a per-column k_index), through the C ABI.

A column applied at k[i] through the sweep handle must equal the same column
applied by a handle built at k[i] alone in a batch of the same width (same
plan, tables and kernels; the sweep gathers the columns of each wavenumber
into one batch, zero-padded to a multiple of 8 columns).  At the
122,880-unknown sphere's 8-point band 0.9 k0 .. 1.1 k0 the sweep must meet
the method's bounds against the FP64 oracle on sampled rows at every
wavenumber (eight rows per wavenumber, relative Frobenius norm over the
columns of that wavenumber): 5e-4 for the FP32 batch (d0 4.5, p 10, one-box
buffer; measured 1.4e-4 .. 3.2e-4 across the band) and 1e-4 for FP64 (d0 4,
p 10, two-box buffer at the two finest levels; measured 1.5e-5 .. 4.3e-5).
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

K0 = 2 * np.pi
ACC32 = dict(d0=5.0, interp_p=10)
BAND32 = dict(d0=4.5, interp_p=10)
BAND64 = dict(d0=4.0, interp_p=10, wide_near=True)


def colerr(a, b):
    return float(np.max(np.linalg.norm(a - b, axis=0) / np.linalg.norm(b, axis=0)))


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    return torch


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_sweep_columns_equal_single_k_handles(torch_cuda, dtype):
    torch = torch_cuda
    from paper_1412_1756_amd import Operator
    V, F = workloads.icosphere(4, 1.0)
    ks = [0.9 * K0, K0, 1.1 * K0]
    sw = Operator(V, F, ks, nlv=4, max_cols=16, **ACC32)
    singles = [Operator(V, F, k, nlv=4, max_cols=16, **ACC32) for k in ks]
    dt = torch.complex64 if dtype == "c64" else torch.complex128
    X = torch.tensor(workloads.cn01_block(sw.N, 12, 40), dtype=dt, device="cuda")
    kidx = np.array([j % 3 for j in range(12)], dtype=np.int32)
    for opname in ("Z", "R", "ZH"):
        Y = sw.apply(X, op=opname, k_index=kidx).cpu().numpy()
        for i, op in enumerate(singles):
            cols = np.nonzero(kidx == i)[0]
            Xp = torch.zeros((X.shape[0], 8), dtype=X.dtype, device="cuda")   # padded to 8 columns
            Xp[:, :len(cols)] = X[:, cols]
            ref = op.apply(Xp, op=opname)[:, :len(cols)].cpu().numpy()
            e = colerr(Y[:, cols], ref)
            print(f"sweep {dtype} op={opname} k={ks[i]:.4f}: {e:.1e}", flush=True)
            assert e == 0.0
    # one wavenumber for the whole batch runs in place
    Y1 = sw.apply(X, k_index=np.full(12, 2, np.int32)).cpu().numpy()
    assert colerr(Y1, singles[2].apply(X).cpu().numpy()) == 0.0
    with pytest.raises(Exception):
        sw.apply(X, k_index=np.full(12, 3, np.int32))


def test_sweep_shared_one_pass_matches_per_wavenumber(torch_cuda):
    """CM_FLAG_SWEEP_SHARED: a Z or Z^H batch spanning several wavenumbers
    runs as one pass (leaf stages per four-column slot, one tree pass over all
    columns with per-slot translators and shift phases).  Each column must
    equal, to FP32 rounding, the same column through a single-wavenumber
    handle with the same discretisation (k_sampling = the largest k, the
    translators truncated at their own k): the two
    routes take the same tables, but the leaf-stage kernels differ (vector
    ALU per slot against the matrix cores), so the sums round differently.
    The bound is three times the distance between the single handle's
    matrix-core and vector-ALU routes (the FP32 rounding scale of this
    operator; measured 2e-5 .. 1.5e-4 across the band, the largest at 0.9 k
    where the sampling of 1.1 k makes the translators large).  Uneven column
    counts per wavenumber go through the gather into slots (padding columns);
    other ops take the per-wavenumber route and match the single handles bit
    for bit."""
    torch = torch_cuda
    from paper_1412_1756_amd import Operator
    V, F = workloads.icosphere(4, 1.0)
    ks = [0.9 * K0, K0, 1.1 * K0]
    sw = Operator(V, F, ks, nlv=4, max_cols=16, sweep_shared=True, **ACC32)
    st = sw.stats()
    assert st["sweep_tables"] == 3 and abs(st["k_sampling"] - ks[2]) < 1e-12
    # single handles with the sweep's discretisation: sampling at the largest
    # k, translators truncated at their own k (sweep_shared with one k)
    same = dict(nlv=4, max_cols=16, k_sampling=ks[2], sweep_shared=True, **ACC32)
    singles = [Operator(V, F, k, **same) for k in ks]
    vec = [Operator(V, F, k, matrix_cores=False, **same) for k in ks]
    X = torch.tensor(workloads.cn01_block(sw.N, 12, 41), dtype=torch.complex64, device="cuda")
    layouts = {"interleaved": np.array([j % 3 for j in range(12)], dtype=np.int32),
               "grouped": np.repeat(np.arange(3, dtype=np.int32), 4),
               "uneven": np.array([0, 0, 0, 0, 0, 1, 1, 2, 2, 2], dtype=np.int32)}
    calls = 0
    for name, kidx in layouts.items():
        Xc = X[:, :len(kidx)].contiguous()
        for opname in ("Z", "ZH", "R"):
            Y = sw.apply(Xc, op=opname, k_index=kidx).cpu().numpy()
            if opname != "R":
                calls += 1
            for i, op in enumerate(singles):
                cols = np.nonzero(kidx == i)[0]
                Xp = torch.zeros((Xc.shape[0], 8), dtype=Xc.dtype, device="cuda")
                Xp[:, :len(cols)] = Xc[:, cols]
                ref = op.apply(Xp, op=opname)[:, :len(cols)].cpu().numpy()
                e = float(np.linalg.norm(Y[:, cols] - ref) / np.linalg.norm(ref))
                if opname == "R":
                    assert e == 0.0
                    continue
                alt = vec[i].apply(Xp, op=opname)[:, :len(cols)].cpu().numpy()
                scale = float(np.linalg.norm(alt - ref) / np.linalg.norm(ref))
                print(f"one-pass sweep {name} op={opname} k={ks[i] / K0:.2f} k0: {e:.1e} "
                      f"(matrix-core vs vector-ALU single handle: {scale:.1e})", flush=True)
                assert e < max(3 * scale, 1e-5)
            assert sw.stats()["sweep_one_pass_calls"] == calls
    # a batch at one wavenumber runs in place through that wavenumber's handle
    Y1 = sw.apply(X, k_index=np.full(12, 1, np.int32)).cpu().numpy()
    assert colerr(Y1, singles[1].apply(X).cpu().numpy()) == 0.0
    assert sw.stats()["sweep_one_pass_calls"] == calls


def test_sweep_shared_sixteen_slots(torch_cuda):
    """The largest one-pass batch: 16 wavenumbers x 4 columns (16 slots, 64
    columns, column j at wavenumber j mod 16); every column against a single
    handle of the same discretisation, to three times the distance between
    that handle's matrix-core and vector-ALU routes (as in the 3-wavenumber
    test)."""
    torch = torch_cuda
    from paper_1412_1756_amd import Operator
    V, F = workloads.icosphere(4, 1.0)
    ks = list(np.linspace(0.9, 1.1, 16) * K0)
    kw = dict(nlv=4, max_cols=64, **ACC32)
    sw = Operator(V, F, ks, sweep_shared=True, **kw)
    X = torch.tensor(workloads.cn01_block(sw.N, 64, 70), dtype=torch.complex64, device="cuda")
    kidx = np.arange(64, dtype=np.int32) % 16
    Y = sw.apply(X, k_index=kidx).cpu().numpy()
    assert sw.stats()["sweep_one_pass_calls"] == 1
    for i in (0, 7, 15):
        same = dict(k_sampling=ks[-1], sweep_shared=True, **kw)
        one, vec = Operator(V, F, ks[i], **same), Operator(V, F, ks[i], matrix_cores=False, **same)
        cols = np.nonzero(kidx == i)[0]
        Xp = torch.zeros((X.shape[0], 8), dtype=X.dtype, device="cuda")
        Xp[:, :len(cols)] = X[:, cols]
        ref = one.apply(Xp)[:, :len(cols)].cpu().numpy()
        alt = vec.apply(Xp)[:, :len(cols)].cpu().numpy()
        e = float(np.linalg.norm(Y[:, cols] - ref) / np.linalg.norm(ref))
        scale = float(np.linalg.norm(alt - ref) / np.linalg.norm(ref))
        print(f"16 slots, k = {ks[i] / K0:.4f} k0: {e:.1e} (matrix-core vs vector-ALU: {scale:.1e})", flush=True)
        assert e < max(3 * scale, 1e-5)


def test_sweep_shared_beyond_sixteen_slots_takes_the_per_wavenumber_route(torch_cuda):
    """A one-pass batch holds at most 16 slots of four columns: 17 wavenumbers
    with one column each take the per-wavenumber route (no one-pass apply),
    whose columns equal single handles of the same discretisation (sampling
    at the largest k, translators truncated at their own k) bit for bit."""
    torch = torch_cuda
    from paper_1412_1756_amd import Operator
    V, F = workloads.icosphere(3, 0.5)
    ks = list(np.linspace(0.9, 1.1, 17) * K0)
    kw = dict(nlv=3, max_cols=32, d0=5.0, interp_p=10)
    sw = Operator(V, F, ks, sweep_shared=True, **kw)
    X = torch.tensor(workloads.cn01_block(sw.N, 17, 60), dtype=torch.complex64, device="cuda")
    kidx = np.arange(17, dtype=np.int32)
    Y = sw.apply(X, k_index=kidx).cpu().numpy()
    assert sw.stats()["sweep_one_pass_calls"] == 0
    for i in (0, 8, 16):
        one = Operator(V, F, ks[i], k_sampling=ks[-1], sweep_shared=True, **kw)
        Xp = torch.zeros((X.shape[0], 8), dtype=X.dtype, device="cuda")
        Xp[:, 0] = X[:, i]
        ref = one.apply(Xp)[:, 0].cpu().numpy()
        assert np.array_equal(Y[:, i], ref), i


@pytest.fixture(scope="module")
def band():
    """The band's wavenumbers and, per wavenumber, eight oracle rows of Z."""
    from oracle import efie
    from oracle.rwg import build_rwg
    V, F, spec = workloads.workload("sphere_r4_n122880")
    ks = list(np.linspace(0.9, 1.1, 8) * K0)
    rng = np.random.default_rng(2)
    geo = efie.Geometry(V, F)
    rwg = build_rwg(V, F)
    rows, Zr = [], []
    for k in ks:
        r = np.sort(rng.choice(len(rwg["edge"]), 8, replace=False))
        rows.append(r)
        Zr.append(efie.rows_Z(V, F, k, r, geo=geo, rwg=rwg))
    return V, F, ks, rows, Zr


def _band_errors(torch, band, acc, ncols, dt, seed, **kw):
    from paper_1412_1756_amd import Operator
    V, F, ks, rows, Zr = band
    print(f"building the 8-wavenumber handle {acc} {kw} (8 plans and near-field fills)", flush=True)
    sw = Operator(V, F, ks, nlv=6, max_cols=ncols, **acc, **kw)
    N = sw.N
    Xh = workloads.cn01_block(N, ncols, seed)
    kidx = np.arange(ncols, dtype=np.int32) % 8
    Y = sw.apply(torch.tensor(Xh, dtype=dt, device="cuda"), k_index=kidx).cpu().numpy()
    errs = []
    for i, k in enumerate(ks):
        cols = np.nonzero(kidx == i)[0]
        ref = Zr[i] @ Xh[:, cols]
        e = float(np.linalg.norm(Y[np.ix_(rows[i], cols)] - ref) / np.linalg.norm(ref))
        errs.append(e)
        print(f"k = {k / K0:.4f} k0: rel err {e:.2e} ({len(rows[i])} rows x {len(cols)} columns)", flush=True)
    return errs


def test_sweep_config4_fp32_batch(torch_cuda, band):
    """A block of 32 right-hand sides, column j at wavenumber j mod 8, FP32
    far field."""
    errs = _band_errors(torch_cuda, band, BAND32, 32, torch_cuda.complex64, 100)
    assert max(errs) < 5e-4


def test_sweep_config4_one_pass(torch_cuda, band):
    """The same block through the one-pass route (CM_FLAG_SWEEP_SHARED: the
    eight wavenumbers sampled at 1.1 k0, each translator truncated by eq. (30)
    at its own k, slots of four columns)."""
    errs = _band_errors(torch_cuda, band, BAND32, 32, torch_cuda.complex64, 100, sweep_shared=True)
    assert max(errs) < 5e-4


def test_sweep_band_fp64(torch_cuda, band):
    """16 right-hand sides (two per wavenumber) in FP64 with the two-box
    buffer."""
    errs = _band_errors(torch_cuda, band, BAND64, 16, torch_cuda.complex128, 200)
    assert max(errs) < 1e-4
