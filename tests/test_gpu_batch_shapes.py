"""The problem shapes of the 64-problem batched workload, run through the library:
2-D N x N slices at 2.08 mm with N radial bins and round(252 N / 344) angles (128 -> 94,
256 -> 188, 344 -> 252), and the mMR slab 344 x 344 x 16 (segments 0, +-1: 24 planes).

* Each problem initialised and run alone matches the FP64 oracle (2-D slices: image
  within 1e-3 after 2 epochs, objective within 1e-4).
* The same problems batched (worker streams, and one HIP graph per batch epoch) give
  bitwise the solo results.

Inputs are generated on the host (NumPy), so the device runs nothing but the library."""
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


# (geometry, subsets, prior, counts, seed)
SPECS = [(synth.slice_2d(128), 8, "tv", 1e5, 18081101),
         (synth.slice_2d(256), 37, "none", 1e6, 18081102),
         (synth.slice_2d(344), 64, "tv", 1e7, 18081103),
         (synth.slab(16), 21, "tv", 3e6, 18081104)]
EPOCHS = 2


def alpha_of(counts):
    return 0.1 * (1e5 / counts) ** 0.5


@pytest.fixture(scope="module")
def problems():
    out = []
    for g, m, prior, counts, seed in SPECS:
        d = synth.brain_problem(g, seed, counts)
        out.append((g, m, prior, counts, seed, d))
    return out


def make(P, g, m, prior, counts, seed, d):
    t = {k: dev(d[k]) for k in ("b", "r", "mult")}
    x = torch.zeros(g.image_shape, dtype=torch.float32, device="cuda:0")
    prm = P.cparams(m, prior, "balanced", True, alpha=alpha_of(counts), seed=seed)
    return P.Reconstruction(g, prm, t["b"], t["r"], t["mult"], x), x


def test_batch_shapes_solo_vs_oracle(P, problems):
    for g, m, prior, counts, seed, d in problems[:3]:
        print(f"[batch-shapes] solo {g.nx}x{g.ny}x{g.nz}, {g.n_ang} angles, m={m}, {prior}",
              flush=True)
        rec, x = make(P, g, m, prior, counts, seed, d)
        rec.epoch(EPOCHS)
        torch.cuda.synchronize()
        prob = S.Problem(g, d["b"], d["r"], d["mult"], n_subsets=m, prior=prior,
                         alpha=alpha_of(counts), sampling="balanced", precond=True)
        st = S.spdhg(prob, EPOCHS * prob.iters_per_epoch(), seed=seed)
        X = prob.reported(st)
        assert rel(x.cpu().numpy(), X[0]) <= 1e-3
        psi_o = prob.objective(X)
        assert abs(float(rec.objective().cpu().numpy()[0]) - psi_o) <= 1e-4 * abs(psi_o)
        rec.close()


@pytest.mark.parametrize("graph", [False, True])
def test_batch_shapes_bitwise_solo(P, problems, graph):
    print(f"[batch-shapes] batch of {len(problems)}, graph={graph}", flush=True)
    solo = []
    for g, m, prior, counts, seed, d in problems:
        rec, x = make(P, g, m, prior, counts, seed, d)
        rec.epoch(EPOCHS)
        torch.cuda.synchronize()
        solo.append(x.cpu().numpy())
        rec.close()
    made = [make(P, *pr) for pr in problems]
    recs = [r for r, _ in made]
    for _ in range(EPOCHS):
        P.batch_epoch(recs, 1, n_streams=4, graph=graph)
        torch.cuda.synchronize()
    for (rec, x), a in zip(made, solo):
        np.testing.assert_array_equal(x.cpu().numpy(), a)
        rec.close()
