"""The no-allocation solve (spp_solve_noalloc) against spp_solve.

Both entry points run the same kernels, so the results must agree bit for
bit (and the FP64 bar of 1e-12 against spp_solve holds a fortiori).  Two calls
in a row share the library's one device scratch, the second with a smaller
grid; a plan whose path needs more than the scratch is refused before
anything is enqueued.
"""
import numpy as np
import pytest

import synthetic

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _err(got, ref):
    return float((got - ref).abs().max().item() / ref.abs().max().item())


def _pair(case):
    import paper_1806_06623_amd as spp
    plan = spp.Plan(case["r_if"], case["th_if"], case["nphi"])
    rho = torch.from_numpy(case["rho"]).to("cuda")
    return plan, rho


def test_noalloc_matches_spp_solve_on_two_calls_in_a_row():
    big = synthetic.stellar_case()                 # fused path, 137.5 MiB of scratch
    small = synthetic.gaussian_blob_case()         # 64 x 32 x 64
    pb, rb = _pair(big)
    ps, rs = _pair(small)
    print(f"[case] noalloc {big['name']} then {small['name']}", flush=True)
    ref_b = pb.solve(rb, G=big["G"])
    ref_s = ps.solve(rs, G=small["G"])
    got_b = pb.solve_noalloc(rb, G=big["G"])
    got_s = ps.solve_noalloc(rs, G=small["G"])     # second call, smaller input, same scratch
    torch.cuda.synchronize()
    eb, es = _err(got_b, ref_b), _err(got_s, ref_s)
    print(f"[parity] noalloc vs spp_solve: {big['name']} {eb:.3e} (bitwise {torch.equal(got_b, ref_b)}), "
          f"{small['name']} {es:.3e} (bitwise {torch.equal(got_s, ref_s)})", flush=True)
    assert eb <= 1e-12 and es <= 1e-12
    assert torch.equal(got_b, ref_b) and torch.equal(got_s, ref_s)
    # the big grid again after the small one: nothing of the earlier calls leaks
    again = pb.solve_noalloc(rb, G=2.0 * big["G"])
    torch.cuda.synchronize()
    assert torch.equal(again, 2.0 * ref_b)


def test_noalloc_refuses_plans_beyond_its_scratch():
    import paper_1806_06623_amd as spp
    # staged path (N_r > 576): two fields of 700 x 64 x 256 doubles, 183.5 MB > 160 MiB
    r_if, th_if, nphi = synthetic.stellar_grid(700, 64, 256)
    plan = spp.Plan(r_if, th_if, nphi)
    rho = torch.zeros((700, 64, 256), dtype=torch.float64, device="cuda")
    with pytest.raises(spp.SphPoissonError) as ei:
        plan.solve_noalloc(rho)
    assert ei.value.status == -2
    assert "scratch" in str(ei.value)
