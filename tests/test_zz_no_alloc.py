"""The no-allocation inner solve (hdgmg_inner_solve_noalloc) through the C ABI.

It must give the results of hdgmg_inner_solve on the same context (same
kernels, same recurrence; only the place of the Krylov scalars and reduction
partials differs), on two calls in a row, the second on a smaller problem,
and call the context's allocator not at all.  Flexible CG (generalized
Stokes) and FGMRES (Oseen, through the same fixed scratch) are both covered.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _solver(n, n_refine, k, **kw):
    import paper_2303_06762_amd as hd
    c, t = synth.kuhn_square(n)
    s = hd.Solver(c, t, n_refine, k, 1.0, 1.0, 1e2, **kw)
    s.assemble()
    return s


def _pair(s, seed):
    b = torch.as_tensor(synth.uniform_pm1(seed, 5, (s.n_skel,)), dtype=torch.float64, device="cuda")
    x_ref, its_ref, rel_ref, st_ref = s.inner_solve(b)
    x = torch.full((s.n_skel,), np.nan, dtype=torch.float64, device="cuda")
    n_live = len(s.allocator.live)
    _, its, rel, st = s.inner_solve_noalloc(b, x)
    torch.cuda.synchronize()
    assert len(s.allocator.live) == n_live, "the no-allocation call allocated"
    return x_ref.cpu().numpy(), its_ref, st_ref, x.cpu().numpy(), its, st


@pytest.mark.parametrize("oseen", [0, 1])
def test_noalloc_matches_inner_solve_two_calls(oseen):
    print(f"no-alloc inner solve, oseen={oseen}: 32x32 k=2 then 8x8 k=1", flush=True)
    kw = dict(oseen=oseen)
    big = _solver(8, 2, 2, **kw)      # 32 x 32 squares, three levels
    small = _solver(4, 1, 1, **kw)    # 8 x 8 squares, two levels
    for s, seed in ((big, 11), (small, 12)):
        x_ref, its_ref, st_ref, x, its, st = _pair(s, seed)
        assert st == st_ref == 0
        assert its == its_ref
        err = np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref)
        print(f"  n_skel={s.n_skel}: its {its} (inner_solve {its_ref}), rel diff {err:.1e}", flush=True)
        assert err <= 1e-12
    big.close()
    small.close()


def test_noalloc_calls_no_allocator():
    print("no-alloc inner solve: allocator callbacks during the call", flush=True)
    s = _solver(4, 2, 2)
    a = s.allocator
    # the context's device allocator is PyTorch's: no new buffer in its
    # bookkeeping and no allocation in the caching allocator's counters
    b = torch.as_tensor(synth.uniform_pm1(3, 5, (s.n_skel,)), dtype=torch.float64, device="cuda")
    x = torch.empty(s.n_skel, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    before = torch.cuda.memory_stats().get("allocation.all.allocated", 0)
    n_live = len(a.live)
    _, its, rel, st = s.inner_solve_noalloc(b, x)
    torch.cuda.synchronize()
    after = torch.cuda.memory_stats().get("allocation.all.allocated", 0)
    assert st == 0 and rel <= 1e-8
    assert len(a.live) == n_live
    assert after == before, (before, after)
    s.close()
