"""Full-size workloads against the oracle: the 256-problem batch and the
two-level AMR hierarchy with a 64^3 base, solved as the benchmark solves them.
At these sizes the oracle does not solve the step itself; it checks the
property that defines the answer at any size: its own residual of the GPU
result, |S - L B_gpu|_2 <= 1.01 rtol |S|_2 with rtol = 1e-10 (the library
stops at rtol on its FP64 residual; 1 % covers the two residual evaluations'
rounding), per problem, on the composite leaf cells for AMR (eqs. 12-14 with
the refluxed coarse-fine faces of section 4)."""
import numpy as np
import pytest

import ohm_inputs as gen
from oracle import amr, ref

from gpu_util import announce, blocks_to_dense, cuda, dense_to_blocks, host

pytestmark = pytest.mark.gpu

RTOL = 1e-10


@pytest.mark.parametrize("precision", [1, 0])
def test_batched256_oracle_residual(precision):
    """256 independent problems (edges 16-64, 2-decade log-normal eta, dt
    10-200x explicit) in one handle, the batched workload's V(4, 4) cycle."""
    import torch
    import paper_1009_0798_amd as ohm
    announce(f"full size: 256 batched problems, precision {precision}")
    probs = gen.config_batched(nprob=256)
    H = ohm.Hierarchy([(p["spec"].base_blocks, p["spec"].dx0, p["spec"].levels) for p in probs])
    B = torch.cat([ohm.to_blocks(torch.from_numpy(p["B"]), p["spec"].levels[0]) for p in probs], dim=1).cuda()
    E = torch.cat([ohm.to_blocks(torch.from_numpy(p["eta"])[None], p["spec"].levels[0]) for p in probs], dim=1).cuda()
    dts = [p["dt"] for p in probs]
    opts = ohm.default_opts(rtol=RTOL, max_iters=200, precision=precision, nu_pre=4, nu_post=4, nu_coarse=1)
    st, stats = ohm.ohm_cn_step(H, [B], [E], dts, opts)
    assert st == 0
    out = host(B)
    announce("full size: 256 batched problems, oracle residuals")
    o, worst = 0, 0.0
    for i, p in enumerate(probs):
        s = p["spec"]
        nb = len(s.levels[0])
        got = blocks_to_dense(out[:, o:o + nb], s.levels[0], s.cells(0))
        o += nb
        S = ref.source(p["B"], p["eta"], s.dx0, p["dt"])
        R = ref.residual(got, S, p["eta"], s.dx0, 0.5 * p["dt"])
        rel = np.linalg.norm(R) / np.linalg.norm(S)
        worst = max(worst, rel)
        assert rel <= 1.01 * RTOL, (i, rel, stats[i])
        # the library's reported residual is the oracle's, to rounding (a
        # problem can converge to the rounding floor, about 1e-16)
        assert abs(rel - stats[i]["rel_res"]) <= 1e-2 * rel + 1e-14, (i, rel, stats[i])
    print("worst oracle rel. residual", worst, "iterations", sorted({s["iters"] for s in stats}))


@pytest.mark.parametrize("precision,cycle", [(0, 1), (1, 1), (0, 0)])
def test_amr2_base64_composite_residual(precision, cycle):
    """The two-level AMR workload at full size (64^3 base, level 1 over the
    central 1/8 plus a seeded 20 % of the other base blocks: 1,232 fine
    blocks), dense-core eta, dt = 20x the fine explicit limit at eta = 10."""
    import paper_1009_0798_amd as ohm
    announce(f"full size: amr2 base 64^3 precision {precision} cycle {cycle}")
    spec = gen.config_amr2(n_base=64, extra_frac=0.2, seed=4)
    assert [len(l) for l in spec.levels] == [512, 1232]
    Bb, eb = gen.amr_fields_fourier(spec, seed=5)
    dt = 20.0 * spec.dx(1) ** 2 / (6 * 10.0)
    H = ohm.Hierarchy([(spec.base_blocks, spec.dx0, spec.levels)])
    Bt = [cuda(b) for b in Bb]
    Et = [cuda(e[None]) for e in eb]
    opts = ohm.default_opts(rtol=RTOL, max_iters=300, precision=precision, cycle=cycle, nu_pre=4, nu_post=4,
                            nu_coarse=1)
    st, stats = ohm.ohm_cn_step(H, Bt, Et, dt, opts)
    print(stats)
    assert st == 0
    C = amr.Composite(spec)
    b = [C.to_dense(l, Bb[l]) for l in range(2)]
    e = [C.to_dense(l, eb[l]) for l in range(2)]
    got = [C.to_dense(l, host(Bt[l])) for l in range(2)]
    S = C.source(b, e, dt)
    R = C.residual(got, S, e, 0.5 * dt)
    rel = np.linalg.norm(C.pack(R)) / np.linalg.norm(C.pack(S))
    print("oracle rel. residual", rel)
    assert rel <= 1.01 * RTOL
    assert abs(rel - stats[0]["rel_res"]) <= 1e-2 * rel + 1e-14
