"""Device primitives against independent host computations (numpy): the complex FP64 MFMA
GEMMs (tiled with composite strides and split K; streaming for K, N <= 64) with conjugation,
batches and grouped problems, the batched FP64 Hermitian eigensolver (Jacobi below n = 32,
Householder + divide and conquer up to n = 256) and the pivoted Cholesky factor."""
import zlib

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2306_14887_amd import bpki as B
    c = B.Context()
    yield c
    c.close()


def _rand(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _ref_gemm(d, A, B, C, nprob, asz, bsz, csz):
    out = C.copy()
    Mi, Ni, Ki = d.get("Mi", d["M"]), d.get("Ni", d["N"]), d.get("Ki", d["K"])
    m = np.arange(d["M"]); n = np.arange(d["N"]); k = np.arange(d["K"])
    am = (m // Mi) * d.get("a_mo", 0) + (m % Mi) * d.get("a_mi", 0)
    ak = (k // Ki) * d.get("a_ko", 0) + (k % Ki) * d.get("a_ki", 0)
    bk = (k // Ki) * d.get("b_ko", 0) + (k % Ki) * d.get("b_ki", 0)
    bn = (n // Ni) * d.get("b_no", 0) + (n % Ni) * d.get("b_ni", 0)
    cm = (m // Mi) * d.get("c_mo", 0) + (m % Mi) * d.get("c_mi", 0)
    cn = (n // Ni) * d.get("c_no", 0) + (n % Ni) * d.get("c_ni", 0)
    alpha = d.get("alpha_re", 1.0) + 1j * d.get("alpha_im", 0.0)
    for p in range(nprob):
        for b in range(d.get("batch", 1)):
            a = A[p * asz:(p + 1) * asz][b * d.get("a_b", 0) + am[:, None] + ak[None, :]]
            bb = B[p * bsz:(p + 1) * bsz][b * d.get("b_b", 0) + bk[:, None] + bn[None, :]]
            if d.get("conjA"): a = a.conj()
            if d.get("conjB"): bb = bb.conj()
            r = alpha * (a @ bb)
            idx = p * csz + b * d.get("c_b", 0) + cm[:, None] + cn[None, :]
            out[idx] = (out[idx] + r) if d.get("beta") else r
    return out


CASES = [
    ("plain_64", dict(M=64, N=64, K=64, a_mi=64, a_ki=1, b_ki=64, b_ni=1, c_mi=64, c_ni=1), 1),
    ("ragged", dict(M=37, N=70, K=19, a_mi=19, a_ki=1, b_ki=70, b_ni=1, c_mi=70, c_ni=1), 1),
    ("kfast_conj", dict(M=96, N=40, K=48, a_mi=1, a_ki=96, b_ki=1, b_ni=48, c_mi=40, c_ni=1,
                        conjA=1, conjB=1), 2),
    ("composite", dict(M=64, Mi=8, N=24, Ni=8, K=32, Ki=4,
                       a_mo=300, a_mi=1, a_ko=16, a_ki=2000,
                       b_ko=200, b_ki=1, b_no=10, b_ni=1000,
                       c_mo=200, c_mi=24, c_no=8, c_ni=1), 3),
    ("batch_beta_alpha", dict(M=16, N=16, K=128, a_mi=128, a_ki=1, b_ki=16, b_ni=1, c_mi=16,
                              c_ni=1, batch=3, a_b=2048, b_b=2048, c_b=256, beta=1,
                              alpha_re=0.5, alpha_im=-2.0), 2),
    ("tiny", dict(M=1, N=2, K=3, a_mi=3, a_ki=1, b_ki=2, b_ni=1, c_mi=2, c_ni=1), 1),
    # long K with few output tiles: split-K path (chunked K, deterministic reduction)
    ("splitk_composite", dict(M=64, N=48, K=4096, Ki=64, a_ko=64 * 64, a_mi=64, a_ki=1,
                              b_ko=64 * 48, b_ki=48, b_ni=1, c_mi=48, c_ni=1, beta=1,
                              alpha_re=-1.5, alpha_im=0.25), 2),
    ("splitk_odd_inner", dict(M=40, N=24, K=700, Ki=7, a_mi=1, a_ko=40 * 7, a_ki=40,
                              b_ko=7, b_ki=1, b_ni=700, c_mi=24, c_ni=1, conjB=1), 1),
    # K, N <= 64 with one stride each and M >= 256: the streaming kernel (B resident in LDS)
    # middle leg of a degree-3 tensor [s][a][b][c] at chi = 22 (K, N not multiples of 16 or 4)
    ("stream_leg_mid", dict(M=22 * 22, Mi=22, N=22, K=22, a_mo=22 * 22, a_mi=1, a_ki=22,
                            b_ki=22, b_ni=1, c_mo=22 * 22, c_mi=1, c_ni=22,
                            batch=2, a_b=22 ** 3, b_b=0, c_b=22 ** 3), 3),
    # last leg at chi = 64 (K unit-stride), accumulate with a complex alpha
    ("stream_leg_last_beta", dict(M=64 * 64, Mi=64, N=64, K=64, a_mo=64 * 64, a_mi=64, a_ki=1,
                                  b_ki=64, b_ni=1, c_mo=64 * 64, c_mi=64, c_ni=1,
                                  batch=2, a_b=64 ** 3, b_b=0, c_b=64 ** 3, beta=1,
                                  alpha_re=0.75, alpha_im=-0.5), 2),
    # ragged M (not a multiple of the 16-row strip), conjugated operands, N < K
    ("stream_ragged_conj", dict(M=1000, N=37, K=61, a_mi=61, a_ki=1, b_ki=1, b_ni=61,
                                c_mi=37, c_ni=1, conjA=1, conjB=1), 2),
    # C unit-stride along M (the transposed-strip variant), ragged M, accumulate
    ("stream_mfast_out", dict(M=1000, N=50, K=64, a_mi=1, a_ki=1000, b_ki=50, b_ni=1,
                              c_mi=1, c_ni=1000, conjB=1, beta=1, alpha_re=-0.5,
                              alpha_im=1.25), 2),
    # K = N = 64 (the fixed-bound variant) with M not a multiple of the 16-row strip (the last
    # strip's rows past M read a clamped row), in both output orientations
    ("stream_full_ragged", dict(M=1000, N=64, K=64, a_mi=64, a_ki=1, b_ki=64, b_ni=1,
                                c_mi=64, c_ni=1, conjA=1, beta=1, alpha_re=0.5,
                                alpha_im=-1.0), 2),
    ("stream_full_ragged_mfast", dict(M=1000, N=64, K=64, a_mi=1, a_ki=1000, b_ki=1, b_ni=64,
                                      c_mi=1, c_ni=1000, conjB=1), 3),
]


def _extent(d, pre):
    Mi = d.get("Mi", d["M"]); Ni = d.get("Ni", d["N"]); Ki = d.get("Ki", d["K"])
    def span(X, Xi, so, si):
        return max(0, X // Xi - 1) * so + (Xi - 1) * si
    if pre == "a":
        e = span(d["M"], Mi, d.get("a_mo", 0), d.get("a_mi", 0)) + span(d["K"], Ki, d.get("a_ko", 0), d.get("a_ki", 0))
        e += (d.get("batch", 1) - 1) * d.get("a_b", 0)
    elif pre == "b":
        e = span(d["K"], Ki, d.get("b_ko", 0), d.get("b_ki", 0)) + span(d["N"], Ni, d.get("b_no", 0), d.get("b_ni", 0))
        e += (d.get("batch", 1) - 1) * d.get("b_b", 0)
    else:
        e = span(d["M"], Mi, d.get("c_mo", 0), d.get("c_mi", 0)) + span(d["N"], Ni, d.get("c_no", 0), d.get("c_ni", 0))
        e += (d.get("batch", 1) - 1) * d.get("c_b", 0)
    return e + 1


@pytest.mark.parametrize("name,desc,nprob", CASES, ids=[c[0] for c in CASES])
def test_gemm_fp32_mode(ctx, name, desc, nprob):
    """FP32 MFMA mode: operands rounded to FP32, FP32 accumulation per K chunk; the error is at
    FP32 level relative to the operand scale."""
    print(f"[gemm fp32] case {name} nprob={nprob}", flush=True)
    rng = np.random.default_rng(zlib.crc32(name.encode()) + 1)
    asz, bsz, csz = _extent(desc, "a"), _extent(desc, "b"), _extent(desc, "c")
    A = _rand(rng, nprob * asz)
    Bm = _rand(rng, nprob * bsz)
    Cm = _rand(rng, nprob * csz)
    got = ctx.test_gemm({**desc, "prec": 1}, A, Bm, Cm, nprob)
    want = _ref_gemm(desc, A, Bm, Cm, nprob, asz, bsz, csz)
    scale = np.sqrt(desc["K"]) * 4 * max(1.0, abs(desc.get("alpha_re", 1)) + abs(desc.get("alpha_im", 0)))
    err = np.abs(got - want).max()
    assert err < 2e-6 * scale
    assert err > 0 or desc["K"] < 4     # really computed in FP32


@pytest.mark.parametrize("name,desc,nprob", CASES, ids=[c[0] for c in CASES])
def test_gemm_matches_numpy(ctx, name, desc, nprob):
    print(f"[gemm] case {name} nprob={nprob}", flush=True)
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    asz, bsz, csz = _extent(desc, "a"), _extent(desc, "b"), _extent(desc, "c")
    A = _rand(rng, nprob * asz)
    Bm = _rand(rng, nprob * bsz)
    Cm = _rand(rng, nprob * csz)
    got = ctx.test_gemm(desc, A, Bm, Cm, nprob)
    want = _ref_gemm(desc, A, Bm, Cm, nprob, asz, bsz, csz)
    scale = np.sqrt(desc["K"]) * 4
    assert np.abs(got - want).max() < 1e-13 * scale


HERM_CASES = [
    # one diagonal tile (the BP closings: 64 x 64 output, K = 2 chi^2 split)
    ("herm_64_splitk", 64, 4096, 2, 0),
    # several tiles: diagonal, lower and (skipped) upper tiles, ragged edge, no split
    ("herm_200", 200, 96, 2, 0),
    ("herm_200_fp32", 200, 96, 1, 1),
    ("herm_128_splitk_fp32", 128, 2048, 2, 1),
]


@pytest.mark.parametrize("name,n,k,nprob,prec", HERM_CASES, ids=[c[0] for c in HERM_CASES])
def test_gemm_hermitian_output(ctx, name, n, k, nprob, prec):
    """herm = 1: C = A A^H computed on the lower triangle and mirrored; equals the full
    product and is exactly Hermitian."""
    print(f"[gemm herm] case {name}", flush=True)
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    # A [n][k] row-major; B = A^H read from the same data: B[kk][j] = conj(A[j][kk])
    d = dict(M=n, N=n, K=k, a_mi=k, a_ki=1, b_ki=1, b_ni=k, c_mi=n, c_ni=1, conjB=1,
             alpha_re=0.75, herm=1, prec=prec)
    A = _rand(rng, nprob * n * k)
    Cm = _rand(rng, nprob * n * n)
    got = ctx.test_gemm(d, A, A, Cm, nprob).reshape(nprob, n, n)
    for p in range(nprob):
        a = A[p * n * k:(p + 1) * n * k].reshape(n, k)
        want = 0.75 * (a @ a.conj().T)
        if prec:
            # FP32 products: relative to the largest entry (the diagonal sums k positive terms)
            assert np.abs(got[p] - want).max() < 1e-6 * np.abs(want).max()
        else:
            assert np.abs(got[p] - want).max() < 1e-13 * np.sqrt(k) * 4
        assert np.array_equal(got[p], got[p].conj().T)


def _c64(x):
    return x.astype(np.complex64).astype(np.complex128)


@pytest.mark.parametrize("store", [5, 3])
@pytest.mark.parametrize("name,desc,nprob", CASES, ids=[c[0] for c in CASES])
def test_gemm_fp32_storage(ctx, name, desc, nprob, store):
    """Operands held in complex FP32 on the device (mixed-precision BP): 5 = A and C (a leg
    absorption into an FP32 buffer), 3 = A and B (a closing into an FP64 message).  Equal to the
    product of the FP32-rounded operands within FP32 accumulation, plus the rounding of an FP32
    output."""
    print(f"[gemm fp32 storage] case {name} store={store}", flush=True)
    rng = np.random.default_rng(zlib.crc32(name.encode()) + 7)
    asz, bsz, csz = _extent(desc, "a"), _extent(desc, "b"), _extent(desc, "c")
    A = _rand(rng, nprob * asz)
    Bm = _rand(rng, nprob * bsz)
    Cm = _rand(rng, nprob * csz)
    got = ctx.test_gemm({**desc, "prec": 1, "store32": store}, A, Bm, Cm, nprob)
    Ar = _c64(A)
    Br = _c64(Bm) if store & 2 else Bm
    Cr = _c64(Cm) if store & 4 else Cm
    want = _ref_gemm(desc, Ar, Br, Cr, nprob, asz, bsz, csz)
    scale = np.sqrt(desc["K"]) * 4 * max(1.0, abs(desc.get("alpha_re", 1)) + abs(desc.get("alpha_im", 0)))
    out_round = 6e-8 * np.abs(want) if store & 4 else 0.0
    assert np.all(np.abs(got - want) < 2e-6 * scale + out_round)


def test_gemm_fp32_storage_hermitian_closing(ctx):
    """The BP closing shape in FP32 storage: C = A A^H (K = 2 chi^2 = 8192 at chi = 64, split K)
    with A and B read as FP32 and the Hermitian FP64 output."""
    print("[gemm fp32 storage] hermitian closing", flush=True)
    rng = np.random.default_rng(3)
    n, k, nprob = 64, 8192, 2
    d = dict(M=n, N=n, K=k, a_mi=k, a_ki=1, b_ki=1, b_ni=k, c_mi=n, c_ni=1, conjB=1,
             herm=1, prec=1, store32=3)
    A = _rand(rng, nprob * n * k)
    got = ctx.test_gemm(d, A, A, np.zeros(nprob * n * n, complex), nprob).reshape(nprob, n, n)
    for p in range(nprob):
        a = _c64(A[p * n * k:(p + 1) * n * k]).reshape(n, k)
        want = a @ a.conj().T
        assert np.abs(got[p] - want).max() < 1e-6 * np.abs(want).max()
        assert np.array_equal(got[p], got[p].conj().T)


def test_gemm_fp32_storage_rejects_other_sets(ctx):
    from paper_2306_14887_amd.bpki import BpkiError
    d = dict(M=64, N=64, K=64, a_mi=64, a_ki=1, b_ki=64, b_ni=1, c_mi=64, c_ni=1)
    z = np.zeros(64 * 64, complex)
    for prec, store in ((1, 1), (1, 7), (0, 5)):
        with pytest.raises(BpkiError):
            ctx.test_gemm({**d, "prec": prec, "store32": store}, z, z, z)


def test_gemm_herm_rejects_invalid_descriptor(ctx):
    from paper_2306_14887_amd.bpki import BpkiError
    d = dict(M=64, N=32, K=64, a_mi=64, a_ki=1, b_ki=32, b_ni=1, c_mi=32, c_ni=1, herm=1)
    with pytest.raises(BpkiError):
        ctx.test_gemm(d, np.zeros(64 * 64, complex), np.zeros(64 * 32, complex),
                      np.zeros(64 * 32, complex))


def test_gemm_rejects_out_of_bounds_descriptor(ctx):
    from paper_2306_14887_amd.bpki import BpkiError
    d = dict(M=64, N=64, K=64, a_mi=64, a_ki=1, b_ki=64, b_ni=1, c_mi=64, c_ni=1)
    A = np.zeros(64 * 64 - 1, complex)            # one element short
    with pytest.raises(BpkiError):
        ctx.test_gemm(d, A, np.zeros(64 * 64, complex), np.zeros(64 * 64, complex))


@pytest.mark.parametrize("n", [1, 2, 5, 16, 31, 32, 40, 63, 64, 65, 97, 127, 128, 129, 200, 256,
                               257, 300, 512])
def test_eigh_matches_numpy(ctx, n):
    print(f"[eigh] n={n}", flush=True)
    rng = np.random.default_rng(n)
    nprob = 6
    X = _rand(rng, nprob, n, n)
    A = X + X.conj().transpose(0, 2, 1)
    # a PSD, rank-deficient problem with a wide spectrum (as in the Gram matrices)
    Y = _rand(rng, n, max(1, n // 3)) * np.logspace(0, -6, max(1, n // 3))[None, :]
    A[1] = Y @ Y.conj().T
    # degenerate spectra: zero, identity, two repeated eigenvalues in a random basis
    A[2] = 0.0
    A[3] = np.eye(n)
    U, _ = np.linalg.qr(_rand(rng, n, n))
    lam = np.where(np.arange(n) < n // 2, 1.0, -0.5)
    A[4] = (U * lam[None, :]) @ U.conj().T
    # a Theta^H Theta-like matrix: rank n/2, singular values from 1 down to 1e-6
    k = max(1, n // 2)
    Y = _rand(rng, 2 * n, k) * np.logspace(0, -6, k)[None, :]
    Y = Y @ _rand(rng, k, n)
    A[5] = Y.conj().T @ Y
    ev, V = ctx.test_eigh(A)
    for p in range(nprob):
        ref = np.sort(np.linalg.eigvalsh(A[p]))[::-1]
        scale = max(np.abs(ref).max(), 1e-300)
        assert np.abs(ev[p] - ref).max() < 1e-13 * scale * max(1, n / 16)
        assert np.all(np.diff(ev[p]) <= 1e-15 * scale)
        # eigenvectors: orthonormal and A V = V diag(ev)
        assert np.abs(V[p].conj().T @ V[p] - np.eye(n)).max() < 1e-12 * max(1, n / 16)
        assert np.abs(A[p] @ V[p] - V[p] * ev[p][None, :]).max() < 1e-12 * scale * max(1, n / 16)


@pytest.mark.parametrize("n,ncols", [(64, 1), (128, 64), (100, 37), (256, 128), (300, 150)])
def test_eigh_leading_columns(ctx, n, ncols):
    """Only the eigenvectors of the ncols largest eigenvalues (the truncation keeps at most chi of
    2 chi): all eigenvalues as with every column, those columns equal to the full solve's, the
    others untouched.  Includes a degenerate spectrum that straddles the cut."""
    print(f"[eigh] n={n} ncols={ncols}", flush=True)
    rng = np.random.default_rng(7 * n + ncols)
    X = _rand(rng, 3, n, n)
    A = X + X.conj().transpose(0, 2, 1)
    U, _ = np.linalg.qr(_rand(rng, n, n))
    lam = np.where(np.arange(n) < ncols + 2, 1.0, np.linspace(0.5, -1.0, n))
    A[1] = (U * lam[None, :]) @ U.conj().T
    k = max(1, n // 2)
    Y = _rand(rng, 2 * n, k) * np.logspace(0, -6, k)[None, :]
    A[2] = (Y @ _rand(rng, k, n)).conj().T @ (Y @ _rand(rng, k, n))
    ev_all, V_all = ctx.test_eigh(A)
    ev, V = ctx.test_eigh(A, ncols=ncols)
    assert np.array_equal(ev, ev_all)
    assert np.array_equal(V[:, :, :ncols], V_all[:, :, :ncols])
    assert not np.any(V[:, :, ncols:])


@pytest.mark.parametrize("n,rank", [(8, 8), (16, 5), (128, 128), (128, 70), (130, 129), (160, 100),
                                    (200, 200), (256, 200), (256, 256), (384, 300),
                                    (512, 512)])
def test_gram_chol(ctx, n, rank):
    """Pivoted Cholesky of A^H A: R^H R = G, and Q = A Wsc is an isometry on the range."""
    print(f"[gram_chol] n={n} rank={rank}", flush=True)
    rng = np.random.default_rng(n + rank)
    nprob = 2
    A = _rand(rng, nprob, 3 * n, rank) @ (_rand(rng, nprob, rank, n) * np.logspace(0, -4, n)[None, None, :])
    G = A.conj().transpose(0, 2, 1) @ A
    R, W = ctx.test_gram_chol(G, 1e-15)
    for p in range(nprob):
        scale = np.abs(G[p]).max()
        assert np.abs(R[p].conj().T @ R[p] - G[p]).max() < 1e-12 * scale
        Q = A[p] @ W[p]
        QQ = Q.conj().T @ Q
        r = int(np.count_nonzero(np.abs(np.diag(QQ)) > 0.5))
        assert r == rank
        idx = np.nonzero(np.abs(np.diag(QQ)) > 0.5)[0]
        assert np.abs(QQ[np.ix_(idx, idx)] - np.eye(r)).max() < 1e-6
        assert np.abs(Q @ R[p] - A[p]).max() < 1e-8 * np.abs(A[p]).max()


def test_mfma_rate_probe(ctx):
    """The MFMA throughput probe returns a rate between a tenth of and the nominal dense peak
    (FP64 78.6, FP32 157.3 TFLOP/s) and rejects bad arguments."""
    from paper_2306_14887_amd import bpki as B
    print("[mfma rate]", flush=True)
    r64 = ctx.test_mfma_rate(0, blocks=512, iters=500)
    r32 = ctx.test_mfma_rate(1, blocks=512, iters=500)
    assert 7.86 < r64 <= 78.6 * 1.02
    assert 15.7 < r32 <= 157.3 * 1.02
    with pytest.raises(B.BpkiError):
        ctx.test_mfma_rate(2)
    with pytest.raises(B.BpkiError):
        ctx.test_mfma_rate(0, blocks=0)


# --- fused BP message (chi = 32 and 64) -----------------------------------------------------------

# (outgoing leg, applied leg, chunk leg) as the BP sweep uses them, site tensors [s][l0][l1][l2]
BP_CLOSE_CASES = [("out0", 0, 2, 1), ("out1", 1, 2, 0), ("out2", 2, 0, 1)]


def _hermitian(rng, n):
    X = _rand(rng, n, n)
    H = X @ X.conj().T
    return H / np.trace(H).real


def _bp_close_case(rng, nprob, o, q, cl, chi):
    """Site tensors T, the chunk leg's message absorbed (Y = T x_cl M_cl), the applied leg's
    message M_q, and the reference message out[b][b'] = sum T M_cl M_q conj(T) over s, a, x."""
    Ts, Ys, Ms, refs = [], [], [], []
    for _ in range(nprob):
        T = _rand(rng, 2, chi, chi, chi) / chi
        Mc, Mq = _hermitian(rng, chi), _hermitian(rng, chi)
        Y = np.moveaxis(np.tensordot(np.moveaxis(T, 1 + cl, -1), Mc, axes=([3], [0])), -1, 1 + cl)
        # views [s][b][a][x] of Y and T
        perm = [0, 1 + o, 1 + q, 1 + cl]
        Yv, Tv = np.transpose(Y, perm), np.transpose(T, perm)
        W = np.tensordot(Yv, Mq, axes=([2], [0]))              # [s][b][x][a]
        ref = np.tensordot(W, np.transpose(Tv, (0, 1, 3, 2)).conj(), axes=([0, 2, 3], [0, 2, 3]))
        Ts.append(T.reshape(-1)); Ys.append(Y.reshape(-1)); Ms.append(Mq); refs.append(ref)
    return np.array(Ys), np.array(Ts), np.array(Ms), np.array(refs)


@pytest.mark.parametrize("chi", [64, 32])
@pytest.mark.parametrize("name,o,q,cl", BP_CLOSE_CASES, ids=[c[0] for c in BP_CLOSE_CASES])
def test_bp_close_matches_numpy(ctx, name, o, q, cl, chi):
    """The fused message of a degree-3 site against numpy complex128, for the three leg
    configurations of the sweep: FP64 MFMA to 1e-12 of the largest entry, FP32 MFMA (FP64 and
    FP32 operand storage) to 2e-5; exactly Hermitian output.  For out0 enough problems that the
    workgroups' chunk runs straddle problems."""
    print(f"[bp_close] {name} chi={chi}", flush=True)
    rng = np.random.default_rng(zlib.crc32(f"{name}{chi}".encode()))
    nprob = (9 if chi == 64 else 20) if name == "out0" else 2
    Y, T, M, ref = _bp_close_case(rng, nprob, o, q, cl, chi)
    stride = (chi * chi, chi, 1)
    st = dict(rs=stride[o], qs=stride[q], cs=stride[cl], ss=chi ** 3)
    scale = np.abs(ref).max()
    got = ctx.test_bp_close(Y, T, M, **st)
    assert np.abs(got - ref).max() < 1e-12 * scale
    assert np.array_equal(got, np.conj(np.transpose(got, (0, 2, 1))))
    for store32 in (0, 1):
        g32 = ctx.test_bp_close(Y, T, M, precision=1, store32=store32, **st)
        err = np.abs(g32 - ref).max() / scale
        print(f"  FP32 store32={store32}: {err:.1e}", flush=True)
        assert 1e-10 < err < 2e-5
        assert np.array_equal(g32, np.conj(np.transpose(g32, (0, 2, 1))))


@pytest.mark.parametrize("chi", [64, 32])
def test_bp_pair_matches_numpy(ctx, chi):
    """The pair closing of a degree-3 site's third message: with Y0 = T x0 M0 and Y1 = T x1 M1 (the
    two summed legs' Hermitian messages absorbed, one in each copy), sum Y0 conj(Y1) over s and
    legs 0, 1 equals sum T M0 M1 conj(T), the message out of leg 2; against numpy complex128 (FP64
    to 1e-12 of the largest entry, FP32 to 2e-5), exactly Hermitian, over enough problems that
    workgroups straddle problems."""
    print(f"[bp_close] pair chi={chi}", flush=True)
    rng = np.random.default_rng(77 + chi)
    nprob = 9 if chi == 64 else 20
    Ys, Ts, refs = [], [], []
    for _ in range(nprob):
        T = _rand(rng, 2, chi, chi, chi) / chi
        M0, M1 = _hermitian(rng, chi), _hermitian(rng, chi)
        Y0 = np.einsum("saxc,ab->sbxc", T, M0)
        Y1 = np.einsum("saxc,xy->sayc", T, M1)
        Z = np.einsum("sbxc,xy->sbyc", Y0, M1)
        refs.append(np.einsum("sbyc,sbyd->cd", Z, T.conj()))
        Ys.append(Y0.reshape(-1)); Ts.append(Y1.reshape(-1))
    Y, T, ref = np.array(Ys), np.array(Ts), np.array(refs)
    M = np.zeros((nprob, chi, chi), complex)
    st = dict(rs=1, qs=chi * chi, cs=chi, ss=chi ** 3, pair=1)
    scale = np.abs(ref).max()
    got = ctx.test_bp_close(Y, T, M, **st)
    assert np.abs(got - ref).max() < 1e-12 * scale
    assert np.array_equal(got, np.conj(np.transpose(got, (0, 2, 1))))
    for store32 in (0, 1):
        g32 = ctx.test_bp_close(Y, T, M, precision=1, store32=store32, **st)
        err = np.abs(g32 - ref).max() / scale
        print(f"  FP32 store32={store32}: {err:.1e}", flush=True)
        assert 1e-10 < err < 2e-5
        assert np.array_equal(g32, np.conj(np.transpose(g32, (0, 2, 1))))


def test_bp_close_rejects_bad_arguments(ctx):
    from paper_2306_14887_amd import bpki as B
    rng = np.random.default_rng(5)
    C = 64
    Y = _rand(rng, 1, 2 * C ** 3)
    M = _rand(rng, 1, C, C)
    with pytest.raises(B.BpkiError):              # reaches past the tensors
        ctx.test_bp_close(Y, Y, M, rs=C * C, qs=1, cs=C, ss=C ** 3 + 1)
    with pytest.raises(B.BpkiError):              # FP32 storage needs FP32 MFMA
        ctx.test_bp_close(Y, Y, M, rs=C * C, qs=1, cs=C, ss=C ** 3, store32=1)
    with pytest.raises(B.BpkiError):              # chi 48 is not built
        ctx.test_bp_close(Y, Y, _rand(rng, 1, 48, 48), rs=48 * 48, qs=1, cs=48, ss=48 ** 3)
    with pytest.raises(B.BpkiError):              # pair is 0 or 1
        ctx.test_bp_close(Y, Y, M, rs=C * C, qs=1, cs=C, ss=C ** 3, pair=2)


@pytest.mark.parametrize("chi", [64, 32])
@pytest.mark.parametrize("o", [0, 1])
def test_bp_close_degree2_matches_numpy(ctx, o, chi):
    """The fused message of a degree-2 site (no chunk leg: the chunks are the two values of s, Y = T):
    out[b][b'] = sum_{s, a, a'} T[s][b][a] M[a][a'] conj(T[s][b'][a']) for both legs against numpy,
    FP64 to 1e-12 and FP32 to 2e-5, on 300 problems (several per workgroup)."""
    print(f"[bp_close] degree 2 leg {o} chi={chi}", flush=True)
    rng = np.random.default_rng(40 + o + chi)
    n = 300
    T = _rand(rng, n, 2, chi, chi) / chi
    M = np.array([_hermitian(rng, chi) for _ in range(n)])
    Tv = T if o == 0 else np.transpose(T, (0, 1, 3, 2))        # [p][s][b][a]
    W = Tv @ M[:, None]                                         # [p][s][b][a']
    ref = np.einsum("psba,psca->pbc", W, Tv.conj())
    st = dict(rs=chi if o == 0 else 1, qs=1 if o == 0 else chi, cs=0, ss=chi * chi, xdim=1)
    Y = T.reshape(n, -1)
    scale = np.abs(ref).max()
    got = ctx.test_bp_close(Y, Y, M, **st)
    assert np.abs(got - ref).max() < 1e-12 * scale
    assert np.array_equal(got, np.conj(np.transpose(got, (0, 2, 1))))
    g32 = ctx.test_bp_close(Y, Y, M, precision=1, store32=1, **st)
    err = np.abs(g32 - ref).max() / scale
    assert 1e-10 < err < 2e-5
