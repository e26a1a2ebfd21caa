"""EM-type updates on the library's projector (eq. MLEM; eq. OSEM on the equidistant-angle
subsets) against the FP64 oracle's osem_step / mlem_step, sub-iteration for
sub-iteration from the same positive start image.  Bar: image within 1e-3 (relative L2)."""
import numpy as np
import pytest

import synth
from oracle import spdhg as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    import paper_1808_07150_amd as lib
    lib.load_library()
    return lib


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda:0")


def rel(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return np.linalg.norm(a - b) / np.linalg.norm(b)


CASES = {
    "slice64": lambda: synth.slice64_problem(),
    "small3d": lambda: synth.brain_problem(
        synth.small_3d(nxy=40, nz=9, n_rad=44, n_ang=24, v=5.0, tan1=0.3), 18081200, 2e5),
    "tall3d": lambda: synth.brain_problem(
        synth.Geometry(nx=40, ny=40, nz=33, vx=5.0, vy=5.0, vz=5.0, n_rad=44, d_rad=5.0,
                       n_ang=24, seg_planes=(33, 29, 29), seg_tan=(0.0, 0.25, -0.25)),
        18081201, 5e5),
    "span11": lambda: synth.brain_problem(synth.mmr(nxy=13, vxy=5.0, n_rad=16, n_ang=6),
                                          18081202, 5e5),
}


@pytest.mark.parametrize("name,m,subiters", [("slice64", 10, 20), ("slice64", 1, 8),
                                             ("small3d", 6, 12), ("tall3d", 4, 8),
                                             ("span11", 3, 6)])
def test_em_parity(P, name, m, subiters):
    print(f"[em] {name} m={m} sub-iterations={subiters}", flush=True)
    d = CASES[name]()
    g = d["geom"]
    prob = S.Problem(g, d["b"], d["r"], d["mult"], n_subsets=m, prior="none")
    u = np.ones(g.image_shape)
    for k in range(subiters):
        u = S.osem_step(prob, u, k % m) if m > 1 else S.mlem_step(prob, u)
    t = {k: dev(d[k]) for k in ("b", "r", "mult")}
    x = torch.ones(g.image_shape, dtype=torch.float32, device="cuda:0")
    rec = P.Reconstruction(g, P.cparams(m, "none", em=True), t["b"], t["r"], t["mult"], x)
    try:
        rec.em_iterate(subiters // 2)
        rec.em_iterate(subiters - subiters // 2)  # continues with the next subset
        torch.cuda.synchronize()
        err = rel(x.cpu().numpy(), u)
        print(f"[em] {name}: rel err {err:.3e}", flush=True)
        assert err <= 1e-3
    finally:
        rec.close()


def test_em_needs_the_flag(P):
    from paper_1808_07150_amd.spdhg import SpdhgError
    d = synth.slice64_problem()
    g = d["geom"]
    t = {k: dev(d[k]) for k in ("b", "r", "mult")}
    x = torch.ones(g.image_shape, dtype=torch.float32, device="cuda:0")
    rec = P.Reconstruction(g, P.cparams(10, "none"), t["b"], t["r"], t["mult"], x)
    try:
        with pytest.raises(SpdhgError) as e:
            rec.em_iterate(1)
        assert e.value.code == -6
    finally:
        rec.close()
