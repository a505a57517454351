"""Matrix-core (MFMA) interpolation/anterpolation against the vector-ALU
kernels and the CPU FP64 oracle, through the C ABI.

Both FP32 paths compute the same sums (the leaf aggregation and
disaggregation, and section III's separable Lagrange interpolation and its
weighted transpose) in a different order, so they differ by FP32 rounding
only: each is measured against the FP64 apply with the same truncation and
interpolation, and the matrix-core path must be about as accurate as the
vector-ALU one (within 50%: the leaf products add four terms per matrix-core
step, and the X part of Z amplifies rounding through near/far cancellation,
4.5e-5 relative to FP64 on this sphere); their mutual difference stays below
1e-4.  Against
the oracle the FP32 bound of the method's product, 5e-4, applies.  Column counts 8, 24 (a partly filled block of column tiles) and 32
with a row stride larger than the column count; the dZ/dk pass exercises the
accumulating (second-term) variants.
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

K0 = 2 * np.pi
ACC32 = dict(d0=5.0, interp_p=10)
TOL_PATH, TOL32 = 1e-4, 5e-4


def colerr(a, b):
    return float(np.max(np.linalg.norm(a - b, axis=0) / np.linalg.norm(b, axis=0)))


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    return torch


@pytest.fixture(scope="module")
def sphere2():
    # radius 2 wavelengths, 30,720 unknowns, 5 levels: interpolation at levels 2 and 3
    V, F = workloads.icosphere(5, 2.0)
    return V, F


@pytest.fixture(scope="module")
def ops(sphere2):
    from paper_1412_1756_amd import Operator
    V, F = sphere2
    mf = Operator(V, F, K0, nlv=5, max_cols=32, **ACC32)
    va = Operator(V, F, K0, nlv=5, max_cols=32, matrix_cores=False, **ACC32)
    return mf, va


@pytest.mark.parametrize("ncols,ld", [(8, 8), (24, 24), (32, 40)])
@pytest.mark.parametrize("opname", ["Z", "R", "X", "ZH"])
def test_mfma_matches_valu(torch_cuda, ops, ncols, ld, opname):
    torch = torch_cuda
    mf, va = ops
    N = mf.N
    print(f"mfma vs valu op={opname} ncols={ncols} ld={ld} N={N}", flush=True)
    Xh = workloads.cn01_block(N, ncols, 300 + ncols)
    buf = torch.zeros((N, ld), dtype=torch.complex64, device="cuda")
    xin = buf[:, :ncols]
    xin.copy_(torch.tensor(Xh, dtype=torch.complex64, device="cuda"))
    o1 = torch.zeros((N, ld), dtype=torch.complex64, device="cuda")[:, :ncols]
    o2 = torch.zeros((N, ld), dtype=torch.complex64, device="cuda")[:, :ncols]
    y1 = mf.apply(xin, op=opname, out=o1).cpu().numpy()
    y2 = va.apply(xin, op=opname, out=o2).cpu().numpy()
    y3 = mf.apply(torch.tensor(Xh, dtype=torch.complex128, device="cuda"), op=opname).cpu().numpy()
    e, e1, e2 = colerr(y1, y2), colerr(y1, y3), colerr(y2, y3)
    print(f"  max column rel diff {e:.2e}; vs fp64: mfma {e1:.2e} valu {e2:.2e}", flush=True)
    assert e < TOL_PATH
    assert e1 <= 1.5 * e2 + 2e-6


def test_mfma_sampled_rows_match_oracle(torch_cuda, sphere2, ops):
    torch = torch_cuda
    from oracle import efie
    V, F = sphere2
    mf, _ = ops
    N = mf.N
    rng = np.random.default_rng(11)
    rows = np.sort(rng.choice(N, 24, replace=False))
    Zr = efie.rows_Z(V, F, K0, rows)
    X = workloads.cn01_block(N, 32, 500)
    Y = mf.apply(torch.tensor(X, dtype=torch.complex64, device="cuda")).cpu().numpy()
    ref = Zr @ X
    e = colerr(Y[rows], ref)
    print(f"mfma fp32 batched vs oracle rows: {e:.3e}", flush=True)
    assert e < TOL32


def test_mfma_dzdk_matches_valu(torch_cuda, sphere2):
    """dZ/dk in FP32 carries a larger rounding error than Z (its far-field
    terms cancel more), so both FP32 paths are measured against the FP64
    apply with the same truncation and interpolation: the matrix-core path
    must be no less accurate than the vector-ALU one, and within the 1e-3
    bound of the FP32 dZ/dk product."""
    torch = torch_cuda
    from paper_1412_1756_amd import Operator
    V, F = sphere2
    mf = Operator(V, F, K0, nlv=5, max_cols=8, deriv=True, **ACC32)
    va = Operator(V, F, K0, nlv=5, max_cols=8, deriv=True, matrix_cores=False, **ACC32)
    X = workloads.cn01_block(mf.N, 8, 700)
    y1 = mf.apply(torch.tensor(X, dtype=torch.complex64, device="cuda"), op="DZDK").cpu().numpy()
    y2 = va.apply(torch.tensor(X, dtype=torch.complex64, device="cuda"), op="DZDK").cpu().numpy()
    y3 = mf.apply(torch.tensor(X, dtype=torch.complex128, device="cuda"), op="DZDK").cpu().numpy()
    e1, e2 = colerr(y1, y3), colerr(y2, y3)
    print(f"dZ/dk vs fp64: mfma {e1:.2e} valu {e2:.2e} (mfma-valu {colerr(y1, y2):.2e})", flush=True)
    assert e1 <= 1.25 * e2 + 1e-6
    assert e1 < 1e-3


def test_near_fp32_option(torch_cuda, sphere2, ops):
    """CM_FLAG_NEAR_FP32: the near-field product from an FP32 copy of the
    values with FP32 accumulation; it may move the FP32 apply by about the
    FP32 rounding of the near part (bound 1e-5 relative), and must keep the
    FP32 accuracy against FP64 (within 25%)."""
    torch = torch_cuda
    from paper_1412_1756_amd import Operator
    V, F = sphere2
    mf, _ = ops
    nf = Operator(V, F, K0, nlv=5, max_cols=32, near_fp32=True, **ACC32)
    Xh = workloads.cn01_block(mf.N, 16, 77)
    X = torch.tensor(Xh, dtype=torch.complex64, device="cuda")
    for opname in ("Z", "R", "X"):
        y1 = mf.apply(X, op=opname).cpu().numpy()
        y2 = nf.apply(X, op=opname).cpu().numpy()
        y3 = mf.apply(torch.tensor(Xh, dtype=torch.complex128, device="cuda"), op=opname).cpu().numpy()
        e, e1, e2 = colerr(y2, y1), colerr(y1, y3), colerr(y2, y3)
        print(f"near fp32 op={opname}: vs c128 near {e:.2e}; vs fp64 {e2:.2e} (c128 near {e1:.2e})", flush=True)
        assert e < 1e-5
        assert e2 <= 1.25 * e1 + 2e-6


def test_mfma_repeat_is_deterministic(torch_cuda, ops):
    torch = torch_cuda
    mf, _ = ops
    X = torch.tensor(workloads.cn01_block(mf.N, 32, 900), dtype=torch.complex64, device="cuda")
    y1 = mf.apply(X).clone()
    y2 = mf.apply(X)
    assert torch.equal(y1, y2)


def test_autotune_choices_and_parity(torch_cuda, sphere2, ops):
    """CM_FLAG_AUTOTUNE: every matrix-core interpolation and anterpolation
    stage gets a timed choice no slower than the default shape, every
    translation level a choice of kernel no slower than the 16-box tiles, and
    the tuned
    product differs from the untuned one by FP32 rounding only (same bounds
    as the matrix-core/vector-ALU comparison), for Z, Z^H and dZ/dk."""
    torch = torch_cuda
    from paper_1412_1756_amd import Operator
    V, F = sphere2
    mf, _ = ops
    at = Operator(V, F, K0, nlv=5, max_cols=32, autotune=True, **ACC32)
    tune = at.stats()["autotune"]
    print("autotune:", tune, flush=True)
    assert {t["stage"] for t in tune} == {"interp_l2", "interp_l3", "anterp_l3", "anterp_l4", "m2l_l2", "m2l_l3",
                                          "m2l_l4"}
    for t in tune:
        if t["stage"].startswith("m2l"):   # translation kernel: 16-box tiles or 64-box shared-source tiles
            assert t["tile"] in (16, 64) and t["ms"] <= t["tile16_ms"]
            continue
        assert t["half_slots"] in (4, 8) and t["row_group"] in (1, 2, 4)
        assert t["default_ms"] < 0 or t["ms"] <= t["default_ms"]
    Xh = workloads.cn01_block(mf.N, 32, 1234)
    X = torch.tensor(Xh, dtype=torch.complex64, device="cuda")
    for opname in ("Z", "ZH"):
        y1 = mf.apply(X, op=opname).cpu().numpy()
        y2 = at.apply(X, op=opname).cpu().numpy()
        y3 = mf.apply(torch.tensor(Xh, dtype=torch.complex128, device="cuda"), op=opname).cpu().numpy()
        e, e1, e2 = colerr(y2, y1), colerr(y1, y3), colerr(y2, y3)
        print(f"autotuned op={opname}: vs untuned {e:.2e}; vs fp64 {e2:.2e} (untuned {e1:.2e})", flush=True)
        assert e < TOL_PATH
        assert e2 <= 1.5 * e1 + 2e-6
    del at
    d1 = Operator(V, F, K0, nlv=5, max_cols=8, deriv=True, **ACC32)
    d2 = Operator(V, F, K0, nlv=5, max_cols=8, deriv=True, autotune=True, **ACC32)
    X8 = torch.tensor(Xh[:, :8], dtype=torch.complex64, device="cuda")
    y1 = d1.apply(X8, op="DZDK").cpu().numpy()
    y2 = d2.apply(X8, op="DZDK").cpu().numpy()
    y3 = d1.apply(torch.tensor(Xh[:, :8], dtype=torch.complex128, device="cuda"), op="DZDK").cpu().numpy()
    e1, e2 = colerr(y1, y3), colerr(y2, y3)
    print(f"autotuned dZ/dk vs fp64 {e2:.2e} (untuned {e1:.2e}); tuned {d2.stats()['autotune']}", flush=True)
    assert e2 <= 1.25 * e1 + 1e-6


def test_interp_theta_tiles_split_over_blocks(torch_cuda):
    """Two 1 x 1 wavelength plates at opposite corners of a 32-wavelength cube
    (8 levels, 0.25-wavelength leaves, 560 unknowns): their only coupling is
    the translation at level 2, whose sampling (L = 109, 110 theta rows) has
    seven theta row tiles, so the matrix-core interpolation into level 2
    splits them over two blocks, and the matrix-core anterpolation out of
    level 2 (110 parent rows per wave in LDS) runs with one wave per block.  The field on plate B from
    sources on plate A against the oracle's Z[B, A] x_A, and the whole
    product against the dense oracle, for the matrix-core and the vector-ALU
    kernels (FP32 bound 5e-4) and the FP64 apply (1e-4; its vector-ALU
    interpolation stages only the child rows each block's parent rows read)."""
    torch = torch_cuda
    from paper_1412_1756_amd import Operator
    from oracle import efie
    V0, F0 = workloads.plate(10, 10, 0.1)
    V = np.vstack([V0 - 15.5, V0 + 15.5])
    F = np.vstack([F0, F0 + len(V0)]).astype(np.int32)
    Z = efie.dense_Z(V, F, K0)
    N = Z.shape[0]
    mf = Operator(V, F, K0, nlv=8, max_cols=8, **ACC32)
    st = {x["l"]: x for x in mf.stats()["levels"]}
    assert st[2]["mf_interp"]["NT"] > 4 and st[2]["far_pairs"] == 2
    e, _ = mf.rwg_table()
    onA = e.max(axis=1) < len(V0)
    Xh = workloads.cn01_block(N, 8, 60)
    Xh[~onA, :] = 0
    ref = Z @ Xh
    refB = ref[~onA]
    va = Operator(V, F, K0, nlv=8, max_cols=8, matrix_cores=False, **ACC32)
    f64 = Operator(V, F, K0, nlv=8, max_cols=8, d0=6.0, interp_p=12)
    y1 = mf.apply(torch.tensor(Xh, dtype=torch.complex64, device="cuda")).cpu().numpy()
    y2 = va.apply(torch.tensor(Xh, dtype=torch.complex64, device="cuda")).cpu().numpy()
    y3 = f64.apply(torch.tensor(Xh, dtype=torch.complex128, device="cuda")).cpu().numpy()
    eB = [colerr(y[~onA], refB) for y in (y1, y2, y3)]
    eAll = [colerr(y, ref) for y in (y1, y2, y3)]
    print(f"plates 32 wl apart: field on B mfma {eB[0]:.2e} valu {eB[1]:.2e} fp64 {eB[2]:.2e}; whole product "
          f"{eAll[0]:.2e} / {eAll[1]:.2e} / {eAll[2]:.2e}; mfma-valu on B {colerr(y1[~onA], y2[~onA]):.2e}", flush=True)
    assert max(eB[:2]) < TOL32 and max(eAll[:2]) < TOL32
    assert eB[2] < 1e-4 and eAll[2] < 1e-4
    assert colerr(y1[~onA], y2[~onA]) < TOL_PATH


def test_batch_of_64_columns_equals_two_of_32(torch_cuda, sphere2):
    """A 64-column batch (the near-field product takes a second column group
    of blocks) gives the same columns, bit for bit, as two 32-column batches
    through the same handle: every kernel treats column tiles independently."""
    torch = torch_cuda
    from paper_1412_1756_amd import Operator
    V, F = sphere2
    op = Operator(V, F, K0, nlv=5, max_cols=64, **ACC32)
    X = torch.tensor(workloads.cn01_block(op.N, 64, 1100), dtype=torch.complex64, device="cuda")
    for opname in ("Z", "R", "X"):
        Y = op.apply(X, op=opname)
        Y1 = op.apply(X[:, :32].contiguous(), op=opname)
        Y2 = op.apply(X[:, 32:].contiguous(), op=opname)
        assert torch.equal(Y[:, :32], Y1) and torch.equal(Y[:, 32:], Y2), opname


def test_concurrent_schedule_equals_sequential(torch_cuda, ops):
    """The apply runs the near field and the translations of levels 3 .. lf
    on two auxiliary streams (joined before their results are read); with
    per-stage timing on it runs everything on the caller's stream in
    dependency order.  Both give the same result bit for bit (FP32 batch and
    FP64 single vector), also over repeated back-to-back applies."""
    torch = torch_cuda
    mf, _ = ops
    for dt, ncols in ((torch.complex64, 32), (torch.complex128, 1)):
        X = torch.tensor(workloads.cn01_block(mf.N, ncols, 950), dtype=dt, device="cuda")
        ys = [mf.apply(X).clone() for _ in range(3)]
        mf.stage_timing(True)
        yt = mf.apply(X).clone()
        mf.stage_timing(False)
        for y in ys:
            assert torch.equal(y, yt)


def test_apply_replays_from_a_captured_graph(torch_cuda, ops):
    """The apply (with its fork/join over the library's streams) captured once
    into a HIP graph through torch.cuda.graph and replayed: every replay, with
    a new input copied into the captured buffer and eager work and
    synchronisations between the replays, equals the eager apply bit for bit
    (FP32 batch and FP64 vector)."""
    torch = torch_cuda
    mf, _ = ops
    for dt, ncols in ((torch.complex64, 32), (torch.complex128, 1)):
        X = torch.zeros((mf.N, ncols), dtype=dt, device="cuda")
        Y = torch.zeros_like(X)
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            mf.apply(X, out=Y, stream=s)            # warm-up outside the capture
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            mf.apply(X, out=Y)
        for seed in (1201, 1202, 1203):
            Xh = torch.tensor(workloads.cn01_block(mf.N, ncols, seed), dtype=dt, device="cuda")
            X.copy_(Xh)
            g.replay()
            torch.cuda.synchronize()
            yg = Y.clone()
            ye = mf.apply(Xh)                       # eager, between the replays
            torch.cuda.synchronize()
            assert torch.equal(yg, ye), (dt, seed)


@pytest.mark.parametrize("ncols,ld", [(8, 8), (16, 16), (32, 40)])
def test_shared_source_translation_equals_tile16(torch_cuda, sphere2, ncols, ld):
    """The 64-box shared-source translation kernels (every variant, forced
    on every level) against the 16-box-tile kernel: every receiver sums its
    sources in the same order, so Z, R, X, Z^H and the dual (dZ/dk) pass
    agree bit for bit."""
    torch = torch_cuda
    from paper_1412_1756_amd import Operator, _lib
    V, F = sphere2
    t16 = Operator(V, F, K0, nlv=5, max_cols=32, deriv=True, **ACC32)
    X = torch.zeros((t16.N, ld), dtype=torch.complex64, device="cuda")
    X[:, :ncols] = torch.tensor(workloads.cn01_block(t16.N, ncols, 700), dtype=torch.complex64)
    X = X[:, :ncols]
    ref = {o: t16.apply(X, o) for o in ("Z", "R", "X", "ZH", "DZDK")}
    for v in (2, 3, 4):
        assert _lib.lib().cm_set_translation_kernel(t16._h, v) == 0
        for o, y in ref.items():
            assert torch.equal(t16.apply(X, o), y), (v, o)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_single_column_translation_equals_tiles(torch_cuda, sphere2, prec):
    """Single-column translations: the receiver-major kernel (default) and
    the 16-box receiver tiles (CM_FLAG_M2L_SINGLE_TILES) sum every
    receiver's sources in increasing source order, so Z, R, X, Z^H and the
    dual (dZ/dk) pass agree bit for bit, also with the two-box buffer, whose
    leaf lists start at distance 3."""
    torch = torch_cuda
    from paper_1412_1756_amd import Operator
    V, F = sphere2
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    for wide in (False, True):
        kw = dict(nlv=5, max_cols=4, deriv=True, wide_near=wide, **ACC32)
        a = Operator(V, F, K0, **kw)
        b = Operator(V, F, K0, m2l_single_tiles=True, **kw)
        x = torch.tensor(workloads.cn01(a.N, 0), dtype=dt, device="cuda")
        for o in ("Z", "R", "X", "ZH", "DZDK"):
            ya, yb = a.apply(x, o), b.apply(x, o)
            assert torch.equal(ya, yb), (prec, wide, o, float((ya - yb).abs().max()))
        del a, b
