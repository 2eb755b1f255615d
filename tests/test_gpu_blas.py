"""GPU parity of the batched complex building blocks (MFMA GEMM, Gauss-Jordan
inverse) against their definitions evaluated in numpy FP64."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _rand(shape, rng, dtype):
    a = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return a.astype(dtype)


def _op(a, op):
    return {0: a, 1: np.swapaxes(a, -1, -2), 2: np.conj(np.swapaxes(a, -1, -2)), 3: np.conj(a)}[op]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("opA,opB", [(0, 0), (1, 0), (0, 1), (2, 3), (3, 2)])
def test_gemm_matches_definition(prec, opA, opB):
    import torch
    from paper_2007_12718_amd import lsh
    rng = np.random.default_rng(opA * 4 + opB)
    dt = np.complex128 if prec == "fp64" else np.complex64
    M, N, K, B = 70, 45, 37, 3
    A = _rand((B, M, K) if opA in (0, 3) else (B, K, M), rng, dt)
    Bm = _rand((B, K, N) if opB in (0, 3) else (B, N, K), rng, dt)
    D = _rand((B, M, N), rng, dt)
    al, be = 0.7 - 0.2j, -0.3 + 1.1j
    tA, tB, tD = (torch.from_numpy(x).cuda() for x in (A, Bm, D))
    C = lsh.dev_gemm(tA, tB, opA, opB, al, be, D=tD).cpu().numpy()
    ref = al * (_op(A.astype(np.complex128), opA) @ _op(Bm.astype(np.complex128), opB)) + be * D
    tol = 1e-13 if prec == "fp64" else 2e-5
    assert np.abs(C - ref).max() <= tol * np.abs(ref).max()


@pytest.mark.parametrize("offset", [0, 1])
@pytest.mark.parametrize("opA", [0, 1, 2, 3])
@pytest.mark.parametrize("opB", [0, 1, 2, 3])
def test_gemm_interior_tiles_every_layout(opA, opB, offset):
    """Every operand form on a product with whole interior tiles and a
    ragged edge in M, N and K, with operands that start 16-byte aligned
    (offset 0) or not (offset 1 element) and odd and even leading dimensions,
    against the definition in FP64."""
    import torch
    from paper_2007_12718_amd import lsh
    rng = np.random.default_rng(16 * opA + 4 * opB + offset)
    M, N, K, B = 197, 131, 263 + offset, 2
    A = _rand((B, M, K) if opA in (0, 3) else (B, K, M), rng, np.complex64)
    Bm = _rand((B, K, N) if opB in (0, 3) else (B, N, K), rng, np.complex64)

    def dev(x):  # a device copy whose data starts `offset` elements into its buffer
        buf = torch.zeros(x.size + offset, dtype=torch.complex64, device="cuda")
        v = buf[offset:].view(x.shape)
        v.copy_(torch.from_numpy(x))
        return v

    C = lsh.dev_gemm(dev(A), dev(Bm), opA, opB, 0.7 - 0.2j).cpu().numpy()
    ref = (0.7 - 0.2j) * (_op(A.astype(np.complex128), opA) @ _op(Bm.astype(np.complex128), opB))
    assert np.abs(C - ref).max() <= 2e-5 * np.abs(ref).max()


@pytest.mark.parametrize("opA,opB", [(0, 0), (0, 1), (2, 3)])
@pytest.mark.parametrize("M,N,K,B", [(300, 379, 502, 1), (128, 70, 1990, 2), (70, 64, 130, 1), (65, 1, 4100, 3),
                                     (300, 379, 100, 1), (4096, 58, 70, 2), (512, 45, 40, 1)])
def test_split_k_gemm_matches_definition(opA, opB, M, N, K, B):
    """Few output tiles: the FP32 product splits K over workgroups (chunks of
    whole K tiles, a ragged last chunk, partial sums reduced with beta D).
    With too little scratch, or K below two K tiles, it is the unsplit kernel."""
    import torch
    from paper_2007_12718_amd import lsh
    rng = np.random.default_rng(M + N + K + opA)
    dt = np.complex64
    A = _rand((B, M, K) if opA in (0, 3) else (B, K, M), rng, dt)
    Bm = _rand((B, K, N) if opB in (0, 3) else (B, N, K), rng, dt)
    D = _rand((B, M, N), rng, dt)
    al, be = 0.7 - 0.2j, -0.3 + 1.1j
    tA, tB, tD = (torch.from_numpy(x).cuda() for x in (A, Bm, D))
    ref = al * (_op(A.astype(np.complex128), opA) @ _op(Bm.astype(np.complex128), opB)) + be * D
    scale = np.sqrt(K) * np.abs(_op(A, opA)).max() * np.abs(_op(Bm, opB)).max() + np.abs(ref).max()
    for ws_bytes in (24 << 20, 16):
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
        C = lsh.dev_gemm(tA, tB, opA, opB, al, be, D=tD, ws=ws).cpu().numpy()
        assert np.abs(C - ref).max() <= 2e-6 * scale, ws_bytes
        C0 = lsh.dev_gemm(tA, tB, opA, opB, al, be, D=tD).cpu().numpy()
        assert np.abs(C - C0).max() <= 2e-6 * scale


def test_gemm_shared_operand_and_large_batch():
    import torch
    from paper_2007_12718_amd import lsh
    rng = np.random.default_rng(5)
    A = _rand((1, 29, 29), rng, np.complex128)
    Bm = _rand((70000, 29, 3), rng, np.complex128)
    C = lsh.dev_gemm(torch.from_numpy(A).cuda(), torch.from_numpy(Bm).cuda()).cpu().numpy()
    idx = [0, 1, 65534, 65535, 69999]
    assert np.abs(C[idx] - A[0] @ Bm[idx]).max() <= 1e-13 * np.abs(C[idx]).max()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("c", [1, 7, 64, 90, 131, 300, 1100, 2100, 3077])
def test_inverse_matches_definition(prec, c):
    """Sizes span the LDS path, one slab, several slabs with a ragged last
    slab and panel, and one to four rows per thread in the panel kernel."""
    import torch
    from paper_2007_12718_amd import lsh
    rng = np.random.default_rng(c)
    dt = np.complex128 if prec == "fp64" else np.complex64
    B = 3 if c < 2000 else 2
    A = _rand((B, c, c), rng, np.complex128) / np.sqrt(c) + 2 * np.eye(c)
    A[1] = A[1][rng.permutation(c)]  # needs row pivoting
    Ai, info = lsh.dev_inverse(torch.from_numpy(A.astype(dt)).cuda())
    assert int(info.abs().sum()) == 0
    ref = np.linalg.inv(A)
    tol = 1e-12 if prec == "fp64" else 5e-5
    assert np.abs(Ai.cpu().numpy() - ref).max() <= tol * np.abs(ref).max() * max(1, np.sqrt(c) / 4)


def test_inverse_reports_singular():
    import torch
    from paper_2007_12718_amd import lsh
    A = np.zeros((2, 8, 8), dtype=np.complex128)
    A[0] = np.eye(8)
    A[1] = np.eye(8)
    A[1, 5, 5] = 0
    _, info = lsh.dev_inverse(torch.from_numpy(A).cuda())
    assert info.cpu().tolist()[0] == 0 and info.cpu().tolist()[1] == 6


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_inverse_reports_singular_blocked(prec):
    """A zero column stays zero under every elimination step, so the first
    zero pivot is at that column (1-based in info).  The singular matrix
    comes first in the batch: the following matrix, stored right after it,
    must come out exact (no write outside the singular matrix's rows)."""
    import torch
    from paper_2007_12718_amd import lsh
    rng = np.random.default_rng(5)
    c = 200
    A = _rand((2, c, c), rng, np.complex128) / np.sqrt(c) + 2 * np.eye(c)
    A[0, :, 150] = 0
    dt = np.complex128 if prec == "fp64" else np.complex64
    Ai, info = lsh.dev_inverse(torch.from_numpy(A.astype(dt)).cuda())
    assert info.cpu().tolist() == [151, 0]
    ref = np.linalg.inv(A[1])
    tol = 1e-12 if prec == "fp64" else 5e-5
    assert np.abs(Ai[1].cpu().numpy() - ref).max() <= tol * np.abs(ref).max() * 4


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("M,N,K,B,opA,opB", [(70, 45, 37, 3, 0, 0), (300, 379, 502, 2, 0, 1), (129, 200, 97, 1, 2, 3),
                                             (64, 64, 64, 5, 1, 0)])
def test_gemm_variants_give_identical_bits(prec, M, N, K, B, opA, opB):
    """Every tile shape and LDS depth adds the same products in the same
    order: the autotuner's choice changes the time, never the result."""
    import torch
    from paper_2007_12718_amd import lsh
    rng = np.random.default_rng(M + N + K)
    dt = np.complex128 if prec == "fp64" else np.complex64
    A = _rand((B, M, K) if opA in (0, 3) else (B, K, M), rng, dt)
    Bm = _rand((B, K, N) if opB in (0, 3) else (B, N, K), rng, dt)
    D = _rand((B, M, N), rng, dt)
    tA, tB, tD = (torch.from_numpy(x).cuda() for x in (A, Bm, D))
    outs = []
    try:
        for v in range(len(lsh.gemm_variants(prec))):
            lsh.gemm_force_variant(v)
            outs.append(lsh.dev_gemm(tA, tB, opA, opB, 0.7 - 0.2j, -0.3 + 1.1j, D=tD).cpu())
    finally:
        lsh.gemm_force_variant(-1)
    for v, C in enumerate(outs):
        assert torch.equal(C, outs[0]), v
    exact = (0.7 - 0.2j) * (_op(A.astype(np.complex128), opA) @ _op(Bm.astype(np.complex128), opB)) + \
        (-0.3 + 1.1j) * D
    tol = 1e-13 if prec == "fp64" else 2e-5
    assert np.abs(outs[0].numpy() - exact).max() <= tol * np.abs(exact).max()


def test_gemm_tuner_records_fastest_variant(tmp_path):
    from paper_2007_12718_amd import lsh
    best, ms = lsh.gemm_tune("fp32", 512, 512, 512, 4, reps=2)
    assert len(ms) == len(lsh.gemm_variants("fp32")) and all(t > 0 for t in ms)
    assert ms[best] == min(ms)
    p = tmp_path / "t.txt"
    lsh.gemm_table_save(p)
    assert lsh.gemm_table_load(p) >= 1
