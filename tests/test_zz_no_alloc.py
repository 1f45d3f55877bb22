"""qsim_probs_noalloc - the float64 reductions of qsim_probs for callers that
cannot allocate device memory, with the partial sums in the library's fixed
device scratch array instead of a workspace - against qsim_probs on the same
amplitudes (two calls in a row, the second on a smaller state, so the
scratch's earlier contents must not leak into the result), and against the
oracle's statistics of those amplitudes."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_1704_01127_amd import qsim
from supremacy_inputs import random_state

pytestmark = pytest.mark.gpu


def noalloc(L, s, out):
    a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    st = L.qsim_probs_noalloc(s.n, s.dt, ctypes.c_void_p(s.amps.data_ptr()), s.amps.numel() * s.amps.element_size(),
                              ctypes.c_void_p(s.stream.cuda_stream), ctypes.c_void_p(out.data_ptr()), s.dt,
                              ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
    assert st == 0, L.qsim_last_error()
    return a.value, b.value, c.value


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_probs_noalloc_matches_probs(dt):
    L = qsim.lib()
    assert L.qsim_noalloc_scratch_bytes() <= 1 << 20
    tdt = torch.float32 if dt == "c64" else torch.float64
    for n, seed in ((22, 11), (15, 12)):  # the second call on a smaller state
        psi = random_state(n, seed)
        s = qsim.State(n, dt, init="keep")
        s.set_amps(torch.from_numpy(psi))
        out_ref = torch.empty(2 ** n, dtype=tdt, device="cuda")
        out_got = torch.full((2 ** n,), -1.0, dtype=tdt, device="cuda")
        ref = s.probs(out_ref)
        got = noalloc(L, s, out_got)
        # the same kernels on the same grid: identical float64 sums and probabilities
        assert got == ref, (n, got, ref)
        assert torch.equal(out_got, out_ref)
        # against the oracle's statistics of the amplitudes the state holds
        held = s.to_numpy().astype(np.complex128)
        on, os2, oent = oracle.stats(held)
        tol_ent = 1e-12 if dt == "c128" else 3e-7  # float states: ln of the mantissa in float
        assert abs(got[0] - on) <= 1e-12 and abs(got[1] - os2) <= 1e-12 * os2 and abs(got[2] - oent) <= tol_ent
        p = out_got.cpu().numpy().astype(np.float64)
        assert np.max(np.abs(p - np.abs(held) ** 2)) <= (1e-15 if dt == "c128" else 2 ** -23 * np.max(p))
        del s
    # the binding's wrapper gives the same, and bad arguments are refused on the host
    s = qsim.State(12, dt, init="uniform")
    assert qsim.probs_noalloc(s.amps) == s.probs()
    dummy = ctypes.c_void_p(s.amps.data_ptr())
    assert L.qsim_probs_noalloc(35, qsim.C64, dummy, 1 << 40, None, None, qsim.C64, None, None, None) == -2
    assert L.qsim_probs_noalloc(12, qsim.C64, None, 1 << 20, None, None, qsim.C64, None, None, None) == -1
    assert L.qsim_probs_noalloc(12, s.dt, dummy, 16, None, None, qsim.C64, None, None, None) == -1
