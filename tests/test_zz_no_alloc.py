"""The allocation-free probability entry point (qs_probs_noalloc) against qs_probs.

Both run the same two kernels with the same grid (the FP64 partial sums of the reduction go to the library's
static device scratch instead of the state's own buffer), so the probabilities and the norm must agree bit for bit.
Two calls in a row, the second on a smaller state, show that the scratch's previous contents never leak into a
result.
"""
import ctypes

import numpy as np
import pytest
import torch

import circuits as C
from paper_2203_16044_amd import binding as B

pytestmark = pytest.mark.gpu


def _noalloc(psi_t, n, dtype, out_t, norm_t):
    L = B.lib()
    f = L.qs_probs_noalloc
    f.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    f.restype = ctypes.c_int
    return f(psi_t.data_ptr() if psi_t is not None else None, n, dtype,
             out_t.data_ptr() if out_t is not None else None, norm_t.data_ptr() if norm_t is not None else None,
             torch.cuda.current_stream().cuda_stream)


def _reference(gpu, n, dtype, psi):
    st = gpu.State(n, dtype)
    st.set(psi)
    P, nrm = st.probs()
    P = P.cpu().numpy().copy()
    st.close()
    return P, nrm


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_noalloc_probs_match_qs_probs_on_two_calls(gpu, dtype):
    qd = B.QS_C128 if dtype == "c128" else B.QS_C64
    tdt = torch.complex128 if dtype == "c128" else torch.complex64
    for n, seed in ((20, 5), (12, 6)):  # the second call is smaller: nothing of the first may leak into it
        psi = C.random_state(n, seed) * 1.3
        ref_P, ref_norm = _reference(gpu, n, dtype, psi)
        buf = torch.as_tensor(psi.astype(np.complex128 if dtype == "c128" else np.complex64)).to("cuda", tdt)
        out = torch.full((1 << n,), -1.0, dtype=torch.float64, device="cuda")
        nrm = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
        assert _noalloc(buf, n, qd, out, nrm) == B.QS_OK, B.lib().qs_last_error()
        torch.cuda.synchronize()
        assert out.cpu().numpy().tobytes() == ref_P.tobytes(), (n, dtype)
        assert float(nrm.item()) == ref_norm, (n, dtype)
        # norm only, then probabilities only
        nrm2 = torch.zeros(1, dtype=torch.float64, device="cuda")
        assert _noalloc(buf, n, qd, None, nrm2) == B.QS_OK
        out2 = torch.zeros(1 << n, dtype=torch.float64, device="cuda")
        assert _noalloc(buf, n, qd, out2, None) == B.QS_OK
        torch.cuda.synchronize()
        assert float(nrm2.item()) == ref_norm
        assert out2.cpu().numpy().tobytes() == ref_P.tobytes()


def test_noalloc_probs_rejects_bad_arguments(gpu):
    buf = torch.zeros(1 << 10, dtype=torch.complex128, device="cuda")
    out = torch.zeros(1 << 10, dtype=torch.float64, device="cuda")
    assert _noalloc(None, 10, B.QS_C128, out, None) == B.QS_EINVAL
    assert _noalloc(buf, 0, B.QS_C128, out, None) == B.QS_EINVAL
    assert _noalloc(buf, B.QS_MAX_QUBITS + 1, B.QS_C128, out, None) == B.QS_EINVAL
    assert _noalloc(buf, 10, 7, out, None) == B.QS_EINVAL
    assert _noalloc(buf, 10, B.QS_C128, None, None) == B.QS_EINVAL
    assert b"NULL" in B.lib().qs_last_error()
    # misaligned amplitude buffer (8 bytes into a complex128 buffer)
    L = B.lib()
    f = L.qs_probs_noalloc
    rc = f(ctypes.c_void_p(buf.data_ptr() + 8), 4, B.QS_C128, ctypes.c_void_p(out.data_ptr()), None,
           ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == B.QS_EINVAL
    torch.cuda.synchronize()
    assert not torch.any(out != 0)  # rejected calls enqueue nothing
