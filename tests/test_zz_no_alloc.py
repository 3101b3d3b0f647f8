"""me_sigma_noalloc (the entry point that allocates nothing, with the library's static scratch)
against me_sigma on the same handle: two calls in a row, the second with a smaller batch, each
compared event by event.  The two share every kernel and the handle's helicity groups, so the
results must be bitwise equal (stronger than the 1e-12 FP64 bar)."""
import pytest

from tests import workloads as W

# (process, precision, first batch, second batch): batches of several chunks of the static
# scratch (gg_ttggg: 64-event chunks in FP64, 128 in the mixed form) and of the handle's chunk
CASES = [
    ("gg_ttgg", "fp64", 100003, 1000),
    ("gg_tt", "mixed_fp16", (1 << 19) + 17, 3000),
    ("gg_tt", "fp64", (1 << 19) + 17, 70001),
    ("gg_ttggg", "fp64", 200, 70),
    ("gg_ttggg", "mixed_bf16", 300, 100),
    ("ee_mumu", "fp64", 8197, 64),
]


@pytest.mark.gpu
@pytest.mark.parametrize("name,precision,n1,n2", CASES)
def test_noalloc_equals_sigma(name, precision, n1, n2):
    import torch
    from paper_2210_11122_amd import Process

    print(f"noalloc {name} {precision} n={n1},{n2}", flush=True)
    proc = Process(name, precision=precision)
    for seed, n in ((11, n1), (12, n2)):
        p = proc.rambo(seed, W.sqrt_s(name), n)
        got = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
        proc.sigma_noalloc(p, got)
        want = proc.sigma(p)
        torch.cuda.synchronize()
        assert torch.isfinite(got).all()
        assert torch.equal(got, want), (name, precision, n, (got - want).abs().max().item())
    proc.close()
