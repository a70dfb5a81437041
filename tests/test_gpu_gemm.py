"""Element-wise parity of the matrix-core product kernels (mpdo_cgemm) with numpy's complex128
matrix product: every contraction of the update runs through them (FP64 and FP32 MFMA on 32 x 32,
64 x 64 and 128 x 128 (FP64: 128 x 64) workgroup tiles, the split-BF16 kernel, k-split partial
sums).

Bars, per element, from the arithmetic: with |X| the matrix of absolute values and
P = |alpha| |op(A)| |op(B)| + |beta| |C0|,

    FP64:   (K + 4) 2^-53 P
    FP32:   (K + 4) 2^-24 P        (operands rounded to FP32, FP32 accumulation over K)
    BF16X3: (3 2^-18 + (K + 4) 2^-24) P   (hi + lo split misses at most 3 2^-18 |a b|)

Shapes cover a single element, ragged edges in every dimension, transposed and conjugated
operands, an output large enough for the 128 x 128 tile, a long k with a small output (k
split), beta != 0 with a complex alpha, and empty products."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_08572_amd import mpdo
    mpdo.load_library()
    return mpdo


def _rand(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _op(X, op):
    return X if op == 0 else (X.T if op == 1 else X.conj().T)


def _unit(prec, mpdo):
    return {mpdo.MPDO_FP64: (0.0, 2.0 ** -53), mpdo.MPDO_FP32: (0.0, 2.0 ** -24),
            mpdo.MPDO_BF16X3: (3 * 2.0 ** -18, 2.0 ** -24)}[prec]


CASES = [
    # M, N, K, op_a, op_b, alpha, beta, split_k
    (1, 1, 1, 0, 0, 1.0, 0.0, False),
    (37, 45, 70, 0, 0, 1.0, 0.0, False),
    (130, 200, 97, 1, 2, 1.0, 0.0, False),
    (130, 200, 97, 2, 1, 0.5 - 0.25j, 1.5j, False),
    (2048, 2048, 96, 0, 0, 1.0, 0.0, False),
    (64, 48, 6000, 2, 0, 1.0, 0.0, True),
    (300, 129, 257, 0, 2, -1.0, 1.0, True),
    (2048, 2048, 96, 1, 2, 0.5 - 0.25j, 1.5j, False),
    (2048, 2048, 200, 2, 0, 1.0, -1.0, True),
    (2048, 2048, 70, 0, 1, 1.0, 0.0, False),
    (768, 768, 8192, 0, 2, 1.0, 0.0, True),
    (768, 77, 8192, 0, 2, 1.0, 0.0, True),
    (768, 768, 8192, 0, 2, 1.0, 0.0, False),
    (2048, 2048, 4096, 0, 0, 1.0, 0.0, False),
    (2100, 1000, 130, 2, 2, 1.0 + 1.0j, 0.5, True),
]


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("prec_name", ["fp64", "fp32", "bf16x3"])
def test_cgemm_elementwise(case, prec_name):
    mpdo = _gpu()
    prec = {"fp64": mpdo.MPDO_FP64, "fp32": mpdo.MPDO_FP32, "bf16x3": mpdo.MPDO_BF16X3}[prec_name]
    M, N, K, oa, ob, alpha, beta, split = CASES[case]
    rng = np.random.default_rng(100 + case)
    A = _rand(rng, (M, K) if oa == 0 else (K, M))
    B = _rand(rng, (K, N) if ob == 0 else (N, K))
    C0 = _rand(rng, (M, N))
    print(f"[gpu] cgemm {prec_name} M={M} N={N} K={K} ops=({oa},{ob}) split={split}", flush=True)
    got = mpdo.cgemm(prec, A, B, oa, ob, alpha, beta, C0, split_k=split)
    ref = alpha * (_op(A, oa) @ _op(B, ob)) + beta * C0
    P = abs(alpha) * (np.abs(_op(A, oa)) @ np.abs(_op(B, ob))) + abs(beta) * np.abs(C0)
    ub, u = _unit(prec, mpdo)
    bar = (ub + (K + 4) * u) * P + 1e-300
    err = np.abs(got - ref)
    print(f"[gpu] max err / bar {float((err / bar).max()):.3f}", flush=True)
    assert np.all(err <= bar), float((err / bar).max())


def test_cgemm_split_bf16_differs_from_fp32():
    """The split-BF16 kernel really ran: on the same product its error is well above FP32's
    (k = 8, so that the FP32 accumulation adds little to either)."""
    mpdo = _gpu()
    rng = np.random.default_rng(7)
    A, B = _rand(rng, (256, 8)), _rand(rng, (8, 256))
    ref = A @ B
    e32 = np.abs(mpdo.cgemm(mpdo.MPDO_FP32, A, B) - ref).max()
    e3 = np.abs(mpdo.cgemm(mpdo.MPDO_BF16X3, A, B) - ref).max()
    print(f"[gpu] max err fp32 {e32:.2e} bf16x3 {e3:.2e}", flush=True)
    assert e3 > 4 * e32


def test_cgemm_empty_and_bad_arguments():
    mpdo = _gpu()
    out = mpdo.cgemm(mpdo.MPDO_FP32, np.zeros((0, 3)), np.zeros((3, 5)))
    assert out.shape == (0, 5)
    C0 = np.ones((2, 2), dtype=complex)
    out = mpdo.cgemm(mpdo.MPDO_FP64, np.zeros((2, 0)), np.zeros((0, 2)), beta=2.0, C0=C0)
    np.testing.assert_array_equal(out, 2.0 * C0)
    with pytest.raises(mpdo.MpdoError):
        mpdo.cgemm(7, np.ones((2, 2)), np.ones((2, 2)))
