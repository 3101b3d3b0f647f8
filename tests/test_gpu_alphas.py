"""GPU per-event strong coupling (me_sigma_alphas) against the oracle evaluated at each
event's own alpha_s (which recomputes every vertex)."""
import numpy as np
import pytest
import torch

import oracle
from tests import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,n", [("ee_mumu", 64), ("gg_tt", 512), ("gg_ttg", 128), ("gg_ttgg", 33),
                                    ("gg_ttggg", 3)])
def test_alphas_per_event_matches_oracle(name, n):
    from paper_2210_11122_amd import Process
    print(f"case alphas {name} n={n}", flush=True)
    p = oracle.rambo(31, W.sqrt_s(name), W.final_masses(name), n)
    a = np.random.default_rng(5).uniform(0.08, 0.2, n)
    proc = Process(name, m_top=W.M_TOP, alpha_em=W.ALPHA_EM, alpha_s=W.ALPHA_S)
    got = proc.sigma_alphas(torch.from_numpy(p).cuda(), torch.from_numpy(a).cuda()).cpu().numpy()
    want = np.array([oracle.me(name, p[e], params=(W.M_TOP, W.ALPHA_EM, a[e])) for e in range(n)])
    rel = np.abs(got / want - 1)
    print(f"{name}: max rel {rel.max():.2e}", flush=True)
    assert rel.max() <= 1e-12


def test_alphas_rejects_host_pointer():
    from paper_2210_11122_amd import Process, binding
    import ctypes
    proc = Process("gg_tt")
    x = torch.zeros((4, 4, 4), dtype=torch.float64, device="cuda")
    out = torch.empty(4, dtype=torch.float64, device="cuda")
    host = np.zeros(4)
    L = binding.load()
    assert L.me_sigma_alphas(proc._h, ctypes.c_void_p(x.data_ptr()), 4, ctypes.c_void_p(host.ctypes.data),
                             ctypes.c_void_p(out.data_ptr()), None) == -1
    assert L.me_sigma_alphas(proc._h, ctypes.c_void_p(x.data_ptr()), 4, None, ctypes.c_void_p(out.data_ptr()),
                             None) == -1
