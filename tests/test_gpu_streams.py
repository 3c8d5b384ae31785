"""An op is read-only after setup, so applies and solves may run on several
streams at once: results must be bitwise those of the same calls one after
another on the current stream (the kernels are deterministic)."""
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dg():
    import torch
    import paper_1711_03590_amd as dg
    assert torch.cuda.is_available()
    dg.lib()
    return dg


def test_concurrent_applies_on_two_streams(dg):
    import torch
    op = dg.Operator((12, 10, 9), 4, curved=True, variable_coef=True)
    adv = dg.AdvectionOperator((12, 10, 9), 4, curved=True)
    u64 = torch.from_numpy(synth.src_vector(op.n_dofs, 61)).cuda()
    u32 = u64.float()
    ref64, ref32, refa = op.apply(u64), op.apply(u32), adv.apply(u64)
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()   # default priority
    outs = []
    s1.wait_stream(torch.cuda.current_stream())
    s2.wait_stream(torch.cuda.current_stream())
    for _ in range(5):
        a, b, c = torch.empty_like(u64), torch.empty_like(u32), torch.empty_like(u64)
        with torch.cuda.stream(s1):
            op.apply(u64, a, stream=s1)
            adv.apply(u64, c, stream=s1)
        with torch.cuda.stream(s2):
            op.apply(u32, b, stream=s2)
        outs.append((a, b, c))
    torch.cuda.synchronize()
    for a, b, c in outs:
        assert torch.equal(a, ref64) and torch.equal(b, ref32) and torch.equal(c, refa)
    op.close()
    adv.close()


def test_solve_on_a_side_stream_is_deterministic(dg):
    import torch
    op = dg.Operator(6, 3, curved=True)
    b = op.rhs()
    torch.cuda.synchronize()
    x0, st0 = op.cg_solve(b, mode=2, rel_tol=1e-10)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        x1 = torch.zeros_like(b)
        x1, st1 = op.cg_solve(b, x1, mode=2, rel_tol=1e-10, stream=s)
    torch.cuda.synchronize()
    assert st0["converged"] and st1["converged"]
    assert st0["iters_inner"] == st1["iters_inner"]
    assert torch.equal(x0, x1)
    op.close()
