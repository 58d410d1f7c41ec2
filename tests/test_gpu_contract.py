"""Pairwise bit-permuted contraction kernels (matnc_contract) vs numpy.

The reference gathers A[m, k], B[k, n] from the flat storage with the stated
bit positions, multiplies in complex128 and scatters C[m, n] back -- a plain
PyTorch/numpy definition of the same operation, independent of the kernels.
"""

import numpy as np
import pytest

from gpu_util import bit_positions_to_index, rel_err, require_gpu, say

pytestmark = pytest.mark.gpu


def make_case(rng, nm, nn, nk, batch):
    ra, rb, rc = nm + nk, nn + nk, nm + nn
    pa = rng.permutation(ra)
    pb = rng.permutation(rb)
    pc = rng.permutation(rc)
    pos = {
        "posA_m": list(pa[:nm]), "posA_k": list(pa[nm:]),
        "posB_k": list(pb[:nk]), "posB_n": list(pb[nk:]),
        "posC_m": list(pc[:nm]), "posC_n": list(pc[nm:]),
    }
    A = (rng.standard_normal((batch, 1 << ra)) + 1j * rng.standard_normal((batch, 1 << ra))).astype(np.complex64)
    Bm = (rng.standard_normal((batch, 1 << rb)) + 1j * rng.standard_normal((batch, 1 << rb))).astype(np.complex64)
    return pos, A, Bm


def reference(pos, A, Bm, nm, nn, nk):
    am = bit_positions_to_index(pos["posA_m"], nm)[:, None] + bit_positions_to_index(pos["posA_k"], nk)[None, :]
    bk = bit_positions_to_index(pos["posB_k"], nk)[:, None] + bit_positions_to_index(pos["posB_n"], nn)[None, :]
    cm = bit_positions_to_index(pos["posC_m"], nm)[:, None] + bit_positions_to_index(pos["posC_n"], nn)[None, :]
    out = np.zeros((A.shape[0], 1 << (nm + nn)), dtype=np.complex128)
    for b in range(A.shape[0]):
        Am = A[b].astype(np.complex128)[am]
        Bk = Bm[b].astype(np.complex128)[bk]
        out[b][cm] = Am @ Bk
    return out


def run(torch, pos, A, Bm, nm, nn, nk, kernel):
    from paper_2212_04749_amd import api
    dev = torch.device("cuda")
    tA = torch.from_numpy(A.view(np.float32).copy()).to(dev)
    tB = torch.from_numpy(Bm.view(np.float32).copy()).to(dev)
    tC = torch.full((A.shape[0], 2 << (nm + nn)), float("nan"), dtype=torch.float32, device=dev)
    keep = api.contract_pair(tA, tB, tC, pos, kernel=kernel)
    torch.cuda.synchronize()
    del keep
    c = tC.cpu().numpy().view(np.complex64)
    return c.astype(np.complex128)


STREAM_CASES = [
    # small K and N: one lane per m, 1 / 2 / 4 m-chunks per lane
    (8, 2, 2, 1), (10, 0, 2, 2), (9, 2, 0, 1), (12, 4, 4, 1), (9, 4, 4, 3), (11, 3, 3, 2),
    # instances below 256 elements
    (5, 3, 2, 7), (3, 1, 1, 33), (0, 2, 3, 5), (7, 4, 1, 3), (14, 2, 3, 1),
    # large K: K split over lane groups
    (2, 3, 6, 4), (8, 2, 11, 3), (0, 0, 10, 4), (10, 1, 7, 2), (4, 3, 9, 5), (9, 0, 6, 2),
    # generic
    (1, 5, 5, 2), (3, 6, 2, 2),
]


@pytest.mark.parametrize("nm,nn,nk,batch", STREAM_CASES)
def test_streaming_kernel(nm, nn, nk, batch):
    torch = require_gpu()
    rng = np.random.default_rng(100 * nm + 10 * nn + nk)
    pos, A, Bm = make_case(rng, nm, nn, nk, batch)
    say(f"stream nm={nm} nn={nn} nk={nk} batch={batch}")
    got = run(torch, pos, A, Bm, nm, nn, nk, 0)
    ref = reference(pos, A, Bm, nm, nn, nk)
    assert rel_err(got, ref) < 2e-6 * max(1.0, np.sqrt(1 << nk))


MFMA_CASES = [(7, 5, 3, 1), (8, 6, 4, 1), (10, 7, 6, 2), (9, 5, 8, 1), (6, 5, 3, 3), (11, 8, 5, 1),
              (8, 8, 10, 1)]


@pytest.mark.parametrize("nm,nn,nk,batch", MFMA_CASES)
def test_mfma_kernel_all_tiles(nm, nn, nk, batch):
    torch = require_gpu()
    from paper_2212_04749_amd import binding as B
    rng = np.random.default_rng(1000 + 100 * nm + 10 * nn + nk)
    pos, A, Bm = make_case(rng, nm, nn, nk, batch)
    ref = reference(pos, A, Bm, nm, nn, nk)
    ran = 0
    for cfg in range(B.matnc_mfma_config_count()):
        say(f"mfma cfg={cfg} nm={nm} nn={nn} nk={nk} batch={batch}")
        try:
            got = run(torch, pos, A, Bm, nm, nn, nk, 100 + cfg)
        except B.MatncError as e:
            assert e.code == B.MATNC_E_INVALID  # tile does not fit
            continue
        ran += 1
        assert rel_err(got, ref) < 2e-6 * max(1.0, np.sqrt(1 << nk)), f"cfg {cfg}"
    assert ran >= 1
