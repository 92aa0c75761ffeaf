"""Checkpoint / resume from the slow-rate filter carry on the GPU.

The model is Markov in the last fast state of each window (eq. h-k-l-2), so the filter state
after window n, (m^f_{n,l}, P^f_{n,l}) = (m_slow[n-1], P_slow[n-1]), is a complete checkpoint:
filtering y[n:] from it as the prior of x_{n+1,0} reproduces the filter outputs of windows n+1..N,
and the log-likelihood splits as log p(y_{1:N}) = log p(y_{1:n}) + log p(y_{n+1:N} | y_{1:n}).
The two runs group the scans differently, so they agree to rounding: states within 1e-9 (float64)
and the float32 tolerance 1e-3, the log-likelihood within 1e-10 and 1e-4 of its magnitude, with
the resumed tail crossing several tiles. The smoother is not resumable (it needs
the future), so only the filter and the log-likelihood are checked.
"""
import numpy as np
import pytest

from paper_2410_00627_amd import workloads as wl
from conftest import assert_close_states

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _srtm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_00627_amd import srtm
    srtm.lib()
    return srtm


CASES = [(4, 2, 20, 3000, 1300, 41), (2, 1, 10, 2100, 257, 42), (6, 1, 5, 1500, 1, 43)]


@pytest.mark.parametrize("nx,ny,L,N,n,seed", CASES, ids=[f"nx{c[0]}ny{c[1]}N{c[3]}n{c[4]}" for c in CASES])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_filter_resumes_from_slow_carry(nx, ny, L, N, n, seed, dtype):
    srtm = _srtm()
    m = wl.random_stable_model(nx, ny, L, seed)
    y = wl.simulate(m, N, seed + 1)
    F, Q, H, R, m0, P0 = srtm.model_tensors(m, "cuda", dtype)
    yt = torch.as_tensor(y, dtype=torch.float64).to("cuda", dtype)
    print(f"[gpu] resume nx={nx} ny={ny} L={L} N={N} at n={n} {dtype}", flush=True)
    full = srtm.filter(F, Q, H, R, L, m0, P0, yt)
    # fresh buffers: the library requires 16-byte aligned arrays, which row slices need not be
    mc, Pc = full["m_slow"][n - 1].clone(), full["P_slow"][n - 1].clone()
    head, rest = yt[:n].clone(), yt[n:].clone()
    tail = srtm.filter(F, Q, H, R, L, mc, Pc, rest)
    torch.cuda.synchronize()
    tol = 1e-9 if dtype == torch.float64 else 1e-3
    g = {k: v.double().cpu().numpy() for k, v in full.items() if k != "info"}
    t = {k: v.double().cpu().numpy() for k, v in tail.items() if k != "info"}
    assert_close_states(t["m_fast"], t["P_fast"], g["m_fast"][n:], g["P_fast"][n:], tol, "resumed fast")
    assert_close_states(t["m_slow"], t["P_slow"], g["m_slow"][n:], g["P_slow"][n:], tol, "resumed slow")
    ll_full = float(srtm.loglik(F, Q, H, R, L, m0, P0, yt))
    ll_head = float(srtm.loglik(F, Q, H, R, L, m0, P0, head))
    ll_tail = float(srtm.loglik(F, Q, H, R, L, mc, Pc, rest))
    ltol = 1e-10 if dtype == torch.float64 else 1e-4
    assert abs(ll_head + ll_tail - ll_full) <= ltol * max(1.0, abs(ll_full)), (ll_head, ll_tail, ll_full)
