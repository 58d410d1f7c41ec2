"""matnc_contract_noalloc (offset tables in the library's static device array)
against matnc_contract (tables in a caller scratch buffer): the same kernels
on the same tables, so the outputs must be identical bit for bit.  Two calls
in a row on one GPU, the second smaller than the first (the array keeps the
first call's tables, which the second must overwrite), for the streaming
kernel and an MFMA tile configuration; both also against the complex128
definition of the pairwise contraction.
"""

import numpy as np
import pytest

from gpu_util import bit_positions_to_index, rel_err, require_gpu, say

pytestmark = pytest.mark.gpu


def _case(rng, nm, nn, nk, batch):
    ra, rb, rc = nm + nk, nn + nk, nm + nn
    pa, pb, pc = rng.permutation(ra), rng.permutation(rb), rng.permutation(rc)
    pos = {"posA_m": list(pa[:nm]), "posA_k": list(pa[nm:]), "posB_k": list(pb[:nk]), "posB_n": list(pb[nk:]),
           "posC_m": list(pc[:nm]), "posC_n": list(pc[nm:])}
    A = (rng.standard_normal((batch, 1 << ra)) + 1j * rng.standard_normal((batch, 1 << ra))).astype(np.complex64)
    B = (rng.standard_normal((batch, 1 << rb)) + 1j * rng.standard_normal((batch, 1 << rb))).astype(np.complex64)
    return pos, A, B


def _reference(pos, A, B, nm, nn, nk):
    am = bit_positions_to_index(pos["posA_m"], nm)[:, None] + bit_positions_to_index(pos["posA_k"], nk)[None, :]
    bk = bit_positions_to_index(pos["posB_k"], nk)[:, None] + bit_positions_to_index(pos["posB_n"], nn)[None, :]
    cm = bit_positions_to_index(pos["posC_m"], nm)[:, None] + bit_positions_to_index(pos["posC_n"], nn)[None, :]
    out = np.zeros((A.shape[0], 1 << (nm + nn)), dtype=np.complex128)
    for b in range(A.shape[0]):
        out[b][cm] = A[b].astype(np.complex128)[am] @ B[b].astype(np.complex128)[bk]
    return out


def _both(torch, pos, A, B, nm, nn, nk, kernel, stream):
    from paper_2212_04749_amd import binding as Bd
    dev = torch.device("cuda")
    tA = torch.from_numpy(A.view(np.float32).copy()).to(dev)
    tB = torch.from_numpy(B.view(np.float32).copy()).to(dev)
    outs = []
    for noalloc in (False, True):
        tC = torch.full((A.shape[0], 2 << (nm + nn)), float("nan"), dtype=torch.float32, device=dev)
        args = (tA.data_ptr(), tB.data_ptr(), tC.data_ptr(), A.shape[0], pos["posA_m"], pos["posA_k"],
                pos["posB_k"], pos["posB_n"], pos["posC_m"], pos["posC_n"], kernel)
        if noalloc:
            Bd.matnc_contract_noalloc(*args, stream.cuda_stream)
            stream.synchronize()
        else:
            scratch = torch.empty(Bd.matnc_contract_scratch_bytes(), dtype=torch.uint8, device=dev)
            torch.cuda.synchronize()
            Bd.matnc_contract(*args, scratch.data_ptr(), scratch.numel(), stream.cuda_stream)
            stream.synchronize()
            del scratch
        outs.append(tC.cpu().numpy())
    return outs


@pytest.mark.parametrize("kernel,first,second", [
    (0, (12, 3, 4, 3), (9, 2, 2, 1)),           # streaming kernel
    (100, (10, 6, 9, 2), (8, 5, 3, 1)),         # MFMA tile configuration 0 (128 x 32)
])
def test_noalloc_matches_scratch_entry_point(kernel, first, second):
    torch = require_gpu()
    rng = np.random.default_rng(4242 + kernel)
    stream = torch.cuda.Stream()
    for nm, nn, nk, batch in (first, second):
        pos, A, B = _case(rng, nm, nn, nk, batch)
        say(f"noalloc kernel {kernel}: m/n/k bits {nm}/{nn}/{nk}, batch {batch}")
        ref_out, got = _both(torch, pos, A, B, nm, nn, nk, kernel, stream)
        assert not np.isnan(got).any()
        assert np.array_equal(got, ref_out), "noalloc output differs from matnc_contract"
        c = got.view(np.complex64).astype(np.complex128)
        assert rel_err(c, _reference(pos, A, B, nm, nn, nk)) < 2e-6 * max(1.0, np.sqrt(1 << nk))


def test_noalloc_rejects_bad_arguments():
    torch = require_gpu()
    from paper_2212_04749_amd import binding as Bd
    x = torch.zeros(64, dtype=torch.float32, device="cuda")
    with pytest.raises(Bd.MatncError) as e:
        Bd.matnc_contract_noalloc(x.data_ptr(), x.data_ptr(), x.data_ptr(), 1, [0], [1], [0], [1], [0, 1], [2],
                                  0, 0)
    assert e.value.code == Bd.MATNC_E_INVALID  # C positions are not a permutation of 0..1
    with pytest.raises(Bd.MatncError) as e:
        Bd.matnc_contract_noalloc(x.data_ptr(), x.data_ptr(), x.data_ptr(), 1, [0], [1], [0], [1], [0], [1],
                                  105, 0)
    assert e.value.code == Bd.MATNC_E_INVALID  # no 128 x 128 tile fits 1-bit operands
