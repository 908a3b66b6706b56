"""The matrix-core DST-I (sine-matrix products on MFMA) and its setup-time choice.

The product pass computes the same transform as the FFT passes, X_k = sum_m x_m
sin(pi k m / N) (the sine diagonalisation of Sec. 2.3), for even N <= 128, as two
half-size products (odd outputs from x_m + x_{N-m}, even outputs from x_m - x_{N-m}).
Variant 4 forces it on every plain pass it supports, so these tests cover it whatever
the setup-time timing would pick:

* every padded half width (16, 32, 48, 64; N = 16 .. 128, full and ragged halves)
  against the oracle's naive sum, on the contiguous axis (ragged row tiles) and on both
  strided axes (ragged column tiles), with 16- and 64-pencil tiles;
* solves through it against the direct oracle solve, mixed against FP64, and a batch;
* the setup-time choice: timed where the operator runs a plain pass of a short axis,
  -1 elsewhere, and reported in the solve statistics.

Tolerances as for the FFT passes (FP64 1e-12 relative to the largest output, FP32
2e-5): the products sum at most 64 terms of unit-bounded weights.
"""
import numpy as np
import pytest

import workloads as W
from oracle import direct, dst as odst

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ah():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2609_16478_amd as mod
    return mod


@pytest.fixture
def gemm(ah):
    ah.set_dst_variant(4)
    yield
    ah.set_dst_variant(0)


def _rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


# half widths H = N/2: 4, 8, 12, 16 (padded to 16), 24, 32 (32), 36, 48 (48), 54, 64 (64)
@pytest.mark.parametrize("N", [8, 16, 24, 32, 48, 64, 72, 96, 108, 128])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_gemm_dst_matches_oracle(ah, gemm, N, prec):
    rng = np.random.default_rng(100 + N)
    p = ah.FP64 if prec == "fp64" else ah.MIXED
    tol = 1e-12 if prec == "fp64" else 2e-5
    # (axis, memory shape): x with 35 and 150 rows (one partial tile; three tiles, the last
    # partial); y with 37 and 70 columns per slab; z with 65 columns
    cases = ((0, (5, 7, N - 1)), (0, (3, 50, N - 1)), (1, (3, N - 1, 37)), (1, (2, N - 1, 70)),
             (2, (N - 1, 5, 13)))
    for axis, shp in cases:
        x = rng.standard_normal(shp)
        xin = x.astype(np.float32).astype(np.float64) if prec == "fp32" else x
        out = ah.dst1(torch.from_numpy(x).cuda(), axis, p).double().cpu().numpy()
        ref = odst.dst1(xin, axis=2 - axis)
        assert _rel(out, ref) < tol, (axis, shp, _rel(out, ref))


@pytest.mark.parametrize("N", [16, 72, 128])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_gemm_dst_large_passes(ah, gemm, N, prec):
    """Passes with at least 512 tiles of 64 pencils (the 64-pencil tile kernels; smaller
    passes use 16-pencil tiles), the last tile partial; compared on sampled slabs."""
    rng = np.random.default_rng(200 + N)
    p = ah.FP64 if prec == "fp64" else ah.MIXED
    tol = 1e-12 if prec == "fp64" else 2e-5
    x = rng.standard_normal((8, 4097, N - 1))  # 32776 rows = 512 tiles + 8 rows
    xin = x.astype(np.float32).astype(np.float64) if prec == "fp32" else x
    out = ah.dst1(torch.from_numpy(x).cuda(), 0, p).double().cpu().numpy()
    for z in (0, 7):
        for sl in (slice(0, 150), slice(4097 - 150, 4097)):
            ref = odst.dst1(xin[z, sl], axis=1)
            assert _rel(out[z, sl], ref) < tol, (z, sl)
    x = rng.standard_normal((600, N - 1, 70))  # 600 slabs x 2 column tiles, the second partial
    xin = x.astype(np.float32).astype(np.float64) if prec == "fp32" else x
    out = ah.dst1(torch.from_numpy(x).cuda(), 1, p).double().cpu().numpy()
    for o in (0, 299, 599):
        ref = odst.dst1(xin[o], axis=0)
        assert _rel(out[o], ref) < tol, o


def test_gemm_dst_involution(ah, gemm):
    # S S = (N/2) I for the DST-I matrix
    for N in (32, 72, 128):
        x = torch.randn(4, 9, N - 1, dtype=torch.float64, device="cuda")
        y = ah.dst1(ah.dst1(x, 0), 0)
        assert torch.allclose(y, x * (N / 2), rtol=0, atol=1e-12 * N)
        y = ah.dst1(ah.dst1(x.transpose(1, 2).contiguous(), 1), 1)
        assert torch.allclose(y, x.transpose(1, 2) * (N / 2), rtol=0, atol=1e-12 * N)


@pytest.mark.parametrize("case", ["c1_32", "cavity_32", "c3_12", "poly3d_8x12x16"])
def test_gemm_solve_matches_direct(ah, gemm, case):
    p = {"c1_32": lambda: W.config1(32), "cavity_32": lambda: W.cavity(32),
         "c3_12": lambda: W.config3(12), "poly3d_8x12x16": lambda: W.poly_exact((8, 12, 16), 3)}[case]()
    U, V, Q, asm = direct.solve(p)
    with ah.Solver(p, tol=1e-14) as s:
        u, v, q, st = s.solve(want_v=True, want_q=True)
    assert st.converged
    assert _rel(u.cpu().numpy(), U) < 1e-12, case
    assert _rel(q.cpu().numpy(), Q) < 1e-10, case


@pytest.mark.parametrize("case", ["c2_64", "c3_16"])
def test_gemm_mixed_matches_fp64(ah, gemm, case):
    p = W.config2(64) if case == "c2_64" else W.config3(16)
    with ah.Solver(p, tol=1e-14) as s:
        u64, *_ = s.solve()
    with ah.Solver(p, precision=ah.MIXED) as s:
        um, _, _, st = s.solve()
    assert st.converged and st.sweeps >= 2
    assert _rel(um.cpu().numpy(), u64.cpu().numpy()) <= 1e-10, (case, st)


def test_gemm_batched_matches_fft(ah):
    """A batch of short 2-D grids (one bucket of repeated grids) with every plain pass on
    the matrix cores, against the FFT passes only: the same solutions to rounding."""
    specs = [sp for sp in W.config4_specs(40, seed=3) if sp["n"] <= 128][:8]
    probs = [W.config4_instance(sp) for sp in specs]
    ah.set_dst_variant(5)
    try:
        ref, st_ref, rc_ref = ah.solve_batched(probs, tol=1e-13)
        ah.set_dst_variant(4)
        outs, st_g, rc = ah.solve_batched(probs, tol=1e-13)
    finally:
        ah.set_dst_variant(0)
    assert rc == ah.OK and rc_ref == ah.OK
    for pb, u, r, s in zip(probs, outs, ref, st_g):
        assert s.converged, pb.name
        assert _rel(u.cpu().numpy(), r.cpu().numpy()) < 1e-11, pb.name


def test_setup_time_kernel_choice(ah):
    """ahoc_setup times the candidate kernels of each plain pass shape and keeps the fastest;
    the statistics report where the matrix-core pass won."""
    ah.set_dst_variant(0)
    # 2-D, x = 64 intervals: the contiguous passes of x are timed; y runs only fused passes
    p = W.manufactured("1 + 0.5*sin(2*pi*x)*cos(2*pi*y)", "sin(pi*x)**2*sin(pi*y)**2", (64, 48),
                       (0.0, 0.0), (1.0, 0.75))
    with ah.Solver(p, tol=1e-12) as s:
        m, tile, td, tg, tb = s.dst_choice(ah.FP64, 0, 0)
        assert m in (0, 1, 2) and td > 0 and tg > 0 and 0 < tb <= min(td, tg)
        assert (m == 2) == (tile > 0)
        assert tb == {0: td, 1: tg}.get(m, tb)
        assert s.dst_choice(ah.FP64, 1, 0)[0] == -1
        assert s.dst_choice(ah.FP64, 0, 1)[0] == -1
        _, _, _, st = s.solve()
        assert st.converged and st.dst_gemm == (1 if m == 1 else 0)
    # 3-D: contiguous x and strided y timed (x = 256 has no matrix-core pass); z only fused
    p = W.poly_exact((256, 24, 16), 3)
    with ah.Solver(p, precision=ah.MIXED) as s:
        mx, _, td, tg, tb = s.dst_choice(ah.MIXED, 0, 0)
        assert mx in (0, 2) and tg == -1 and 0 < tb <= td
        my, _, td, tg, tb = s.dst_choice(ah.MIXED, 1, 1)
        assert my in (0, 1, 2) and td > 0 and tg > 0 and 0 < tb <= min(td, tg)
        assert s.dst_choice(ah.MIXED, 2, 1)[0] == -1
        _, _, _, st = s.solve()
        assert st.converged and st.dst_gemm == (8 if my == 1 else 0)
    # a second handle with the same shapes makes the same choices (kept for the process)
    with ah.Solver(p, precision=ah.MIXED) as s:
        assert s.dst_choice(ah.MIXED, 0, 0)[0] == mx and s.dst_choice(ah.MIXED, 1, 1)[0] == my
    # forced or disabled selections are not timed
    ah.set_dst_variant(5)
    try:
        with ah.Solver(W.config1(32), tol=1e-12) as s:
            assert s.dst_choice(ah.FP64, 0, 0) == (-1, 0, -1.0, -1.0, -1.0)
    finally:
        ah.set_dst_variant(0)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_tuned_one_tile_solves_match_default(ah, prec):
    """Solves whose plain passes run the one-tile kernels at every tile the tuner may pick
    (through the explicit-tile override) agree with the default kernels to rounding."""
    p = ah.FP64 if prec == "fp64" else ah.MIXED
    pb = W.config3(32)
    ah.set_dst_variant(5)
    try:
        with ah.Solver(pb, precision=p, tol=1e-12) as s:
            ref, *_ = s.solve()
        for tile in (1, 2, 4, 8, 16):
            for kind in (0, 1):
                ah.set_dst_tile(kind, p, tile)
            try:
                with ah.Solver(pb, precision=p, tol=1e-12) as s:
                    u, _, _, st = s.solve()
            except ah.AhocError:
                continue  # a tile the kernel cannot launch at this length
            finally:
                for kind in (0, 1):
                    ah.set_dst_tile(kind, p, 0)
            assert st.converged
            assert _rel(u.cpu().numpy(), ref.cpu().numpy()) < 1e-10, tile
    finally:
        ah.set_dst_variant(0)
