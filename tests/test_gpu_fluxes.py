"""GPU parity of the face fluxes of grad Phi (spp_face_fluxes) against the oracle.

Inputs are seeded synthetic fields or the oracle's own solutions; nothing the
oracle sees comes from the HIP path.  Interior faces: both sides take the same
FP64 difference of Phi and multiply it by geometric factors computed in a
different order, so they agree to a few ulps of each flux; the bar is
|F_gpu - F_oracle| <= 1e-13 |F_oracle| element by element.  The outer boundary
face goes through the modal transform of the outermost shell on both sides; the
bar there is 1e-12 of the shell's largest flux (the FP64 solve tolerance).
"""
import ctypes

import numpy as np
import pytest

import synthetic
from oracle import fluxes, spectral

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_INTERIOR = 1e-13
TOL_OUTER = 1e-12


def _gpu_fluxes(r_if, th_if, nphi, phi, path=None):
    import paper_1806_06623_amd as spp
    plan = spp.Plan(r_if, th_if, nphi)
    if path is not None:
        plan.path = path
    x = torch.from_numpy(np.ascontiguousarray(phi)).to("cuda")
    F = plan.face_fluxes(x)
    torch.cuda.synchronize()
    return [f.cpu().numpy() for f in F]


def _compare(name, got, ref):
    Fr, Ft, Fp = ref
    gr, gt, gp = got
    worst = 0.0
    for g, f, tag in ((gr[:-1], Fr[:-1], "r"), (gt, Ft, "theta"), (gp, Fp, "phi")):
        assert np.all(np.isfinite(g)), tag
        e = np.abs(g - f)
        bad = e > TOL_INTERIOR * np.abs(f) + 1e-300
        worst = max(worst, float(np.max(e / np.maximum(np.abs(f), 1e-300))))
        assert not bad.any(), f"{name} {tag}: {int(bad.sum())} elements, first at {np.argwhere(bad)[0]}"
    eo = float(np.max(np.abs(gr[-1] - Fr[-1])) / np.max(np.abs(Fr[-1])))
    print(f"[flux] {name}: interior max rel {worst:.2e}, outer face {eo:.2e}", flush=True)
    assert eo <= TOL_OUTER, f"{name} outer face: {eo}"
    assert np.all(gt[:, -1, :] == 0.0)


def test_fluxes_of_the_solution_gaussian_blob():
    c = synthetic.gaussian_blob_case()
    print(f"[case] {c['name']} fluxes of the oracle solution", flush=True)
    phi = spectral.solve(c["r_if"], c["th_if"], c["nphi"], c["rho"], c["G"])
    got = _gpu_fluxes(c["r_if"], c["th_if"], c["nphi"], phi)
    _compare(c["name"], got, fluxes.face_fluxes(c["r_if"], c["th_if"], c["nphi"], phi))


@pytest.mark.parametrize("nr,nth,nphi,seed,uniform_theta,r0", [
    (37, 6, 8, 1, True, 0.0),      # rows not a multiple of the 8-row chunk, plane of 48 (< one block)
    (2, 4, 4, 2, True, 0.0),       # smallest grid of the fused path
    (2, 2, 4, 3, True, 0.0),       # smallest grid (staged path only: N_theta = 2)
    (40, 24, 16, 4, False, 0.0),   # non-uniform theta, plane of 384 (a block and a half)
    (17, 128, 256, 5, True, 0.0),  # full angular grid, one row past a chunk (XCD-ordered plane blocks)
    (5, 3, 2048, 6, True, 0.0),    # largest N_phi
    (12, 8, 16, 7, False, 2.0),    # inner boundary at r = 2 (zero-flux face, not stored)
    (6, 200, 8, 8, True, 0.0),     # N_theta = 200: outer-term products over 7 partial 32-column blocks
])
def test_fluxes_of_random_fields(nr, nth, nphi, seed, uniform_theta, r0):
    rng = np.random.default_rng(seed)
    r_if = np.concatenate(([r0], r0 + np.cumsum(rng.uniform(0.3, 1.7, nr))))
    if uniform_theta:
        th_if = synthetic.theta_interfaces(nth)
    else:
        th_if = np.concatenate(([0.0], np.sort(rng.uniform(0.1, np.pi - 0.1, nth - 1)), [np.pi]))
    phi = rng.standard_normal((nr, nth, nphi))
    print(f"[case] random field {nr}x{nth}x{nphi} seed {seed}", flush=True)
    got = _gpu_fluxes(r_if, th_if, nphi, phi)
    _compare(f"random_{nr}x{nth}x{nphi}", got, fluxes.face_fluxes(r_if, th_if, nphi, phi))


def test_fluxes_do_not_depend_on_the_solve_path():
    """The flux kernel reads the plan's tables only; a plan forced onto the
    staged path gives the same fluxes."""
    c = synthetic.stellar_case(nr=48, nth=16, nphi=32, seed=9)
    phi = np.random.default_rng(9).standard_normal((48, 16, 32))
    a = _gpu_fluxes(c["r_if"], c["th_if"], c["nphi"], phi)
    b = _gpu_fluxes(c["r_if"], c["th_if"], c["nphi"], phi, path="staged")
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_gauss_law_and_sampled_parity_at_full_size():
    """550 x 128 x 256 stellar workload, launched as the benchmark does:
    fluxes of the oracle's solution; every outer-face flux and 4096 sampled
    interior fluxes per direction against the oracle, and the outer faces
    summing to 4 pi G M."""
    c = synthetic.stellar_case()
    print(f"[case] {c['name']} full size", flush=True)
    phi = spectral.solve(c["r_if"], c["th_if"], c["nphi"], c["rho"], c["G"])
    got = _gpu_fluxes(c["r_if"], c["th_if"], c["nphi"], phi)
    ref = fluxes.face_fluxes(c["r_if"], c["th_if"], c["nphi"], phi)
    rng = np.random.default_rng(17)
    idx = tuple(rng.integers(0, n, 4096) for n in phi.shape)
    ridx = (np.minimum(idx[0], phi.shape[0] - 2),) + idx[1:]
    for g, f, at, tag in ((got[0], ref[0], ridx, "r"), (got[1], ref[1], idx, "theta"), (got[2], ref[2], idx, "phi")):
        e = np.abs(g[at] - f[at])
        assert np.all(e <= TOL_INTERIOR * np.abs(f[at]) + 1e-300), tag
    eo = float(np.max(np.abs(got[0][-1] - ref[0][-1])) / np.max(np.abs(ref[0][-1])))
    assert eo <= TOL_OUTER, eo
    r_if, th_if, nphi = c["r_if"], c["th_if"], c["nphi"]
    dV = np.outer((r_if[1:] ** 3 - r_if[:-1] ** 3) / 3.0, np.cos(th_if[:-1]) - np.cos(th_if[1:])) * (2 * np.pi / nphi)
    mass = float(np.sum(c["rho"] * dV[:, :, None]))
    total = float(np.sum(got[0][-1]))
    print(f"[flux] full size: outer face {eo:.2e}; total outer flux / 4 pi G M - 1 = "
          f"{total / (4 * np.pi * c['G'] * mass) - 1:.2e}", flush=True)
    assert abs(total - 4 * np.pi * c["G"] * mass) <= 1e-11 * 4 * np.pi * c["G"] * mass


def test_argument_errors_enqueue_nothing():
    import paper_1806_06623_amd as spp
    from paper_1806_06623_amd._binding import lib
    plan = spp.Plan(np.array([0.0, 1.0, 2.0]), synthetic.theta_interfaces(4), 4)
    phi = torch.zeros(plan.shape, dtype=torch.float64, device="cuda")
    fr, ft, fp = (torch.empty_like(phi) for _ in range(3))
    vp = ctypes.c_void_p
    ws = vp(plan.workspace.data_ptr())
    s = vp(torch.cuda.current_stream().cuda_stream)
    ptr = lambda t: vp(t.data_ptr())
    assert lib.spp_face_fluxes(plan._plan, ptr(phi), ptr(fr), ptr(ft), None, ws, s) == -1      # NULL
    assert lib.spp_face_fluxes(plan._plan, ptr(phi), ptr(fr), ptr(fr), ptr(fp), ws, s) == -1   # overlap
    assert lib.spp_face_fluxes(plan._plan, ptr(phi), ptr(fr), ptr(ft), ptr(phi), ws, s) == -1  # alias of phi
    assert lib.spp_face_fluxes(plan._plan, vp(phi.data_ptr() + 8), ptr(fr), ptr(ft), ptr(fp), ws, s) == -1   # misaligned phi
    assert lib.spp_face_fluxes(plan._plan, ptr(phi), ptr(fr), ptr(ft), ptr(fp), vp(ws.value + 64), s) == -1   # misaligned workspace
    assert lib.spp_face_fluxes(plan._plan, ptr(phi), ptr(fr), ptr(ft), ptr(fp), ptr(fp), s) == -1   # workspace on a flux field
    assert lib.spp_face_fluxes(plan._plan, ptr(phi), ptr(fr), ptr(ft), ptr(fp), ws, s) == 0
    torch.cuda.synchronize()


def test_face_fluxes_replay_in_a_hip_graph():
    """The call allocates nothing and records no memset, so a caller may
    capture it: three replays of a captured call, with eager work on the
    device between them, each equal bit for bit to the eager call."""
    import paper_1806_06623_amd as spp
    c = synthetic.stellar_case(nr=48, nth=32, nphi=64, seed=13)
    plan = spp.Plan(c["r_if"], c["th_if"], c["nphi"])
    phi = torch.from_numpy(np.random.default_rng(13).standard_normal((48, 32, 64))).to("cuda")
    ref = [f.clone() for f in plan.face_fluxes(phi)]          # eager (also warms the launch caches)
    out = tuple(torch.full_like(phi, float("nan")) for _ in range(3))
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.face_fluxes(phi, out=out)
    for rep in range(3):
        for o in out:
            o.fill_(float("nan"))
        scratch = torch.randn(1 << 20, device="cuda", dtype=torch.float64)
        scratch.mul_(2.0)                                      # eager work between replays
        g.replay()
        torch.cuda.synchronize()
        for o, r in zip(out, ref):
            assert torch.equal(o, r), f"replay {rep}"


def test_binding_rejects_wrong_buffers_before_launching():
    """Output tensors and workspaces the caller passes are checked by the
    binding (the C ABI sees plain pointers and cannot): wrong shape, dtype or
    size raises ValueError and nothing is enqueued."""
    import paper_1806_06623_amd as spp
    plan = spp.Plan(np.array([0.0, 1.0, 2.0, 3.0]), synthetic.theta_interfaces(8), 16)
    phi = torch.zeros(plan.shape, dtype=torch.float64, device="cuda")
    good = tuple(torch.empty_like(phi) for _ in range(3))
    small_ws = torch.empty(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(ValueError):
        plan.face_fluxes(phi, out=(good[0], good[1], torch.empty(7, dtype=torch.float64, device="cuda")))
    with pytest.raises(ValueError):
        plan.face_fluxes(phi, out=(good[0], good[1], good[2].float()))
    with pytest.raises(ValueError):
        plan.face_fluxes(phi, workspace=small_ws)
    with pytest.raises(ValueError):
        plan.solve(phi, out=torch.empty((2, 8, 16), dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        plan.solve(phi, workspace=small_ws)
    with pytest.raises(ValueError):
        plan.solve_mixed(phi, workspace=small_ws)
    torch.cuda.synchronize()
