"""The scratch lifetime calls of the boundary: me_reserve_scratch allocates up front what every
call of at most n events on a stream needs, so such calls allocate nothing more;
me_release_scratch waits for the stream and frees it; me_scratch_bytes reports what a handle
holds.  Later calls allocate again and give bitwise the same results."""
import pytest
import torch

from tests import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,precision,piped", [("gg_ttg", "fp64", False), ("gg_ttgg", "mixed_fp16", False),
                                                  ("gg_ttggg", "fp64", True)])
def test_reserve_then_release(name, precision, piped):
    from paper_2210_11122_amd import Process
    p = Process(name, m_top=W.M_TOP, alpha_em=W.ALPHA_EM, alpha_s=W.ALPHA_S, precision=precision)
    chunk = p.info["chunk_events"]
    # a piped call (more than one chunk of a process with partial slots) also uses the two
    # internal streams of the caller's stream
    n = 2 * chunk + 5 if piped else min(chunk, 5000) + 3
    print(f"scratch lifetime: {name} {precision} n={n} chunk={chunk}", flush=True)
    x = p.rambo(W.SEED, W.sqrt_s(name), n)
    y1 = torch.empty(n, dtype=torch.float64, device="cuda")
    y2 = torch.empty(n, dtype=torch.float64, device="cuda")
    y3 = torch.empty(n // 3, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    base = p.scratch_bytes()
    p.reserve_scratch(n, stream=s)
    held = p.scratch_bytes()
    assert held > base
    # a reservation of fewer events changes nothing
    p.reserve_scratch(n // 2, stream=s)
    assert p.scratch_bytes() == held
    p.sigma(x, out=y1, stream=s)
    p.sigma(x[: n // 3].contiguous(), out=y3, stream=s)
    s.synchronize()
    assert p.scratch_bytes() == held, "a call within the reservation allocated"
    p.release_scratch(stream=s)
    assert p.scratch_bytes() == base
    p.release_scratch(stream=s)          # nothing left to free
    assert p.scratch_bytes() == base
    p.sigma(x, out=y2, stream=s)         # allocates again, on demand
    s.synchronize()
    assert p.scratch_bytes() > base
    assert torch.equal(y1, y2)
    assert torch.equal(y3, y1[: n // 3])
    assert bool(torch.isfinite(y1).all()) and bool((y1 > 0).all())
    p.release_scratch(stream=s)
    assert p.scratch_bytes() == base
