"""Plan uploads: the host-written part of a plan's workspace is assembled in a
pooled pinned buffer at creation and copied by the plan's first ray trace, on
that call's stream.

Plans created back to back while the default stream is still busy (more
pending plans than the pool keeps, so the pool must grow), then traced and
filled on a non-blocking stream, must give bit-identical D to the same plans
created and run one at a time.
"""
import numpy as np
import pytest

import fspb_inputs as fi

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _problems(n):
    out = []
    for k in range(n):
        g = fi.slab_phantom(200 + k, n=(24 + k, 20, 16), spacing=(0.5, 0.5, 0.5), lung_side=(2, 5),
                            bone_side=(1, 2))
        beams = fi.coplanar_beams(3, (0.1, -0.05, 0.0), 100.0, 1.0, 1.0, 3, 3, step_deg=70.0)
        out.append(fi.Problem(f"upload{k}", g, beams, fi.default_kernel(k + 1)))
    return out


def _host(csr):
    return (csr.indptr.cpu().numpy().copy(), csr.indices.cpu().numpy().copy(),
            csr.values.cpu().numpy().copy())


def test_back_to_back_plans_on_a_side_stream(torch_gpu):
    torch = torch_gpu
    from paper_0908_4417_amd import Plan
    probs = _problems(11)
    dens = [torch.from_numpy(np.ascontiguousarray(p.grid.density, dtype=np.float32)).to("cuda:0")
            for p in probs]
    ref = []
    for p, d in zip(probs, dens):
        plan = Plan(p, "cuda:0", density=d)
        ref.append(_host(plan.compute()))
        del plan
    torch.cuda.synchronize()

    # keep the default stream busy, then create every plan (their copies queue behind)
    a = torch.full((4096, 4096), 1.0 / 4096, device="cuda:0")
    for _ in range(6):
        a = a @ a
    plans = [Plan(p, "cuda:0", density=d) for p, d in zip(probs, dens)]
    side = torch.cuda.Stream()
    got = []
    with torch.cuda.stream(side):
        for plan in plans:
            got.append(plan.compute(stream=side))
    side.synchronize()
    torch.cuda.synchronize()
    for k, (r, g) in enumerate(zip(ref, got)):
        g = _host(g)
        assert np.array_equal(r[0], g[0]), f"plan {k}: row pointers differ"
        assert np.array_equal(r[1], g[1]), f"plan {k}: columns differ"
        assert np.array_equal(r[2], g[2]), f"plan {k}: values differ"
    assert float(a[0, 0]) == pytest.approx(1.0 / 4096, rel=1e-3)
