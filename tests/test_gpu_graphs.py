"""HIP-graph replay of the CG chunks (tc_set_launch use_graphs = 1): the
replayed launches are the direct launches captured once, so a batch stepped
with graphs ends bitwise equal to the same batch stepped without them."""
import numpy as np
import pytest

from gpu_util import log, tc
from workloads import scenes

pytestmark = pytest.mark.gpu


def _run(envs, use_graphs, steps=4):
    ctx = tc.Context(0)
    ctx.set_launch(use_graphs=use_graphs)
    pads = []
    for e in envs:
        m = e.pad.material
        pads.append(tc.Pad(ctx, e.pad.X, e.pad.tets, dict(E=m.E, nu=m.nu, density=m.density),
                           tc.make_params(precision="mixed", dt=e.params.dt, dhat=e.params.dhat,
                                          kappa=e.params.kappa, newton_tol=e.params.newton_tol,
                                          cg_rel_tol=0.2, cg_eta_max=0.2, cg_forcing=2)))
    stats = []
    for s in range(1, steps + 1):
        st = tc.step_batch(ctx, pads, [[e.pose(s)] for e in envs])
        stats.append([(x.status, x.newton_iters, x.cg_iters) for x in st])
    out = [(p.read("positions"), p.read("sigma")) for p in pads]
    for p in pads:
        p.close()
    ctx.close()
    return stats, out


def test_graph_replay_bitwise_equal_to_direct_launches():
    b60 = scenes.config3()
    envs = [scenes.config1(), b60[0], b60[5]]
    st_d, out_d = _run(envs, 0)
    st_g, out_g = _run(envs, 1)
    log(f"direct {st_d}\ngraphs {st_g}")
    assert st_d == st_g
    for (xd, sd), (xg, sg) in zip(out_d, out_g):
        assert np.array_equal(xd, xg) and np.array_equal(sd, sg)
