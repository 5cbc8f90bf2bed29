"""GPU parity of the batched V-cycle and the block preconditioners against the oracle.

Same colour order on both sides; double V-cycles to 1e-11 relative, float
V-cycles to 2e-5 relative (single-precision rounding through the cycle).
"""

import numpy as np
import pytest
import torch

import sg_inputs
from gpu_util import note, rel_max, to_dev, to_host
from oracle import mg, precond, system

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,width,colour,nu,coarsest,a0", [
    (128, 35, "four", (2, 2), 8, False),
    (64, 21, "four", (1, 1), 8, True),
    (128, 20, "rb", (1, 1), 8, False),
    (32, 6, "four", (2, 2), 32, False),
    (16, 1, "rb", (2, 1), 4, True),
    (256, 126, "four", (2, 2), 8, True),     # row-phase smoother, two waves per node
    (128, 64, "four", (1, 3), 8, False),     # odd sweep counts (ping-pong ends in the second buffer)
    (256, 210, "four", (2, 2), 8, False),    # all P modes at once (B_D width)
    (128, 6, "four", (2, 2), 8, False),      # narrow row-phase smoother (lanes over rows and modes)
    (256, 21, "four", (1, 2), 8, True),
    (256, 1, "four", (2, 2), 8, False),
    (128, 8, "four", (2, 1), 8, True),       # tile cycle of a few modes (float), uneven sweep counts
    (256, 3, "four", (1, 2), 8, False),
])
def test_vcycle_matches_oracle(n, width, colour, nu, coarsest, a0):
    import paper_1304_1755_amd as sgbt
    note(f"vcycle n={n} width={width} {colour} {nu} coarsest={coarsest}")
    a0n = sg_inputs.a0_noise_field(n) if a0 else None
    # the V-cycle work space holds up to P columns: m = 4, p = 3 (P = 35) or m = 6, p = 4 (P = 210)
    m, p = (4, 3) if width <= 35 else (6, 4)
    g = sgbt.Problem(n, m, p, 0.3, a0_nodal=a0n, colour=colour, nu1=nu[0], nu2=nu[1], coarsest=coarsest)
    o = system.build_problem(n, m, p, 0.3, a0_nodal=a0n)
    H = mg.Hierarchy(o.K[0], n, coarsest=coarsest, colour_mode=colour, nu1=nu[0], nu2=nu[1])
    f = sg_inputs.uniform_block(g.N, width, seed=11)
    ref = H.vcycle(f)
    u = to_host(g.vcycle(to_dev(f)))
    assert rel_max(u, ref) < 1e-11
    u32 = to_host(g.vcycle(to_dev(f, torch.float32), prec=1))
    assert rel_max(u32, ref) < 2e-5
    g.close()


@pytest.mark.parametrize("cfg,kind", [("c2", "tri"), ("c2", "diag"), ("c3_65", "tri"), ("c5", "tri")])
def test_preconditioners_match_oracle(cfg, kind):
    import paper_1304_1755_amd as sgbt
    note(f"precond {kind} {cfg}")
    c = sg_inputs.CONFIGS[cfg]
    a0 = sg_inputs.a0_noise_field(c["n"]) if cfg == "c5" else None
    g = sgbt.Problem(c["n"], c["m"], c["p"], c["sigma"], c["corr_len"], a0_nodal=a0)
    o = system.build_problem(c["n"], c["m"], c["p"], c["sigma"], c["corr_len"], a0_nodal=a0)
    H = mg.Hierarchy(o.K[0], c["n"], coarsest=8)
    R = sg_inputs.uniform_block(g.N, g.P, seed=21)
    fn = precond.precond_tri if kind == "tri" else precond.precond_diag
    ref = fn(o, R.T, H.vcycle).T
    Z = to_host(g.precond(to_dev(R), kind=kind))
    assert rel_max(Z, ref) < 1e-11
    Zm = to_host(g.precond(to_dev(R), kind=kind, prec=2))
    assert rel_max(Zm, ref) < 5e-5
    g.close()


def test_vcycle_width_above_P_is_rejected():
    import paper_1304_1755_amd as sgbt
    g = sgbt.Problem(16, 2, 1, 0.3)
    f = torch.zeros((g.N, g.P + 1), dtype=torch.float64, device="cuda")
    with pytest.raises(sgbt.SGError) as e:
        g.vcycle(f)
    assert e.value.code == sgbt.SG_EINVAL
    g.close()


def test_exact_inner_solves_make_bt_the_block_lower_solve():
    import scipy.sparse.linalg as spla
    import paper_1304_1755_amd as sgbt
    note("precond tri exact inner c1")
    c = sg_inputs.CONFIGS["c1"]
    g = sgbt.Problem(c["n"], c["m"], c["p"], c["sigma"], c["corr_len"], coarsest=c["n"])
    o = system.build_problem(c["n"], c["m"], c["p"], c["sigma"], c["corr_len"])
    R = sg_inputs.uniform_block(g.N, g.P, seed=5)
    BT = precond.assemble_BT(o)
    ref = spla.spsolve(BT.tocsc(), R.T.ravel()).reshape(o.P, o.N).T
    Z = to_host(g.precond(to_dev(R), kind="tri"))
    assert rel_max(Z, ref) < 1e-11
    g.close()
