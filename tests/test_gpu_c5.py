"""GPU parity at the multi-boson workload's full size: the 64^4 lattice in 4096 blocks Omega of 8^4
(inner Lambda_0 of 6^4, 1040 boundary sites each), 12 boson fields (N = 24, c = 0.5), links and
fields drawn on the GPU (seeds 5101-5103), with the library's default field grouping (as many
fields per block solve as fit in memory).

* eq. (localMB): S^a of sampled blocks against the oracle (FP64 solves of the same sources) to
  1e-9 relative, for the FP32-inner default and the plain FP64 form; all 49 152 pairs at FP64 true
  relative residual <= 1e-10;
* the block solutions of the sampled blocks (dd_block_solve over the whole lattice, four fields a
  call) against the oracle's solves to 1e-8, and their true residuals recomputed by the oracle.
"""
import numpy as np
import pytest

import synth
from oracle import mb, roots, wilson

pytestmark = pytest.mark.gpu

L = (64, 64, 64, 64)
KAPPA = 0.1365
NF = 12
S = 4096
NBD = 1040
SAMPLE = [0, 1, 1365, 2730, 4095]


@pytest.fixture(scope="module")
def c5():
    from paper_2211_06902_amd import dd

    ctx = dd.Context(0)
    blk = ctx.make_blocks(L, -1, [[8] * 8] * 4, inner_d=1)
    U = synth.gauge_field_device(L, 0.2, 5101)
    g = ctx.load_gauge(blk, U, "f32")
    U_host = U.cpu().numpy()
    del U
    chi = synth.spinor_field_device(NF, blk.total_bnd_sites, 5102)
    xi = synth.spinor_field_device(NF, blk.total_sites, 5103)
    u = dd.mb_roots(2 * NF, 0.5)
    tab = blk.tables()
    yield dict(dd=dd, ctx=ctx, blk=blk, g=g, U=U_host, chi=chi, xi=xi, u=u, boxes=tab[0][:, :8],
               inner=tab[0][:, 8:16])
    g.close()
    blk.close()
    ctx.close()


def test_c5_geometry(c5):
    blk = c5["blk"]
    assert blk.n_blocks == 4096 and blk.total_sites == 64**4 and blk.total_bnd_sites == 4096 * NBD
    assert np.all(c5["inner"] == [1, 1, 1, 1, 6, 6, 6, 6])
    assert np.allclose(c5["u"], roots.mb_roots(2 * NF, 0.5)[:NF], rtol=0, atol=1e-15)


def _oracle_action(c5, blocks):
    bx = c5["boxes"][blocks]
    inner = c5["inner"][blocks]
    chi = np.concatenate([c5["chi"][:, b * NBD:(b + 1) * NBD].cpu().numpy() for b in blocks], axis=1)
    xi = np.concatenate([c5["xi"][:, b * S:(b + 1) * S].cpu().numpy() for b in blocks], axis=1)
    return mb.mb_local_action(L, -1, KAPPA, c5["U"], bx, inner, c5["u"], chi, xi, tol=1e-12)[0]


@pytest.mark.parametrize("inner_prec", ["f32", "f64"])
def test_c5_multiboson_action_matches_oracle(c5, inner_prec):
    dd = c5["dd"]
    Sb, tot, info, st = c5["ctx"].multiboson_action(c5["blk"], c5["g"], KAPPA, c5["u"], c5["chi"], c5["xi"],
                                                     params=dd.solve_params(inner_prec=inner_prec))
    assert st == dd.DD_OK
    assert info["true_relres"].shape == (NF, 4096)
    assert np.all(info["true_relres"] <= 1e-10)
    Sb = Sb.cpu().numpy()
    assert np.all(np.isfinite(Sb)) and np.all(Sb > 0)
    assert abs(tot - Sb.sum()) <= 1e-12 * Sb.sum()
    ref = _oracle_action(c5, SAMPLE)
    rel = np.abs(Sb[SAMPLE] - ref) / ref
    print("S^a of blocks %s: max relative difference to the oracle %.2e" % (SAMPLE, rel.max()))
    assert rel.max() <= 1e-9


def test_c5_block_solutions_match_oracle(c5):
    import torch

    dd = c5["dd"]
    xi = c5["xi"]
    x = torch.empty_like(xi)
    for f0 in range(0, NF, 4):
        _, info, st = c5["ctx"].block_solve(c5["blk"], c5["g"], KAPPA, xi[f0:f0 + 4], x[f0:f0 + 4],
                                            params=dd.solve_params(inner_prec="f32"))
        assert st == dd.DD_OK and np.all(info["true_relres"] <= 1e-10)
    bx = c5["boxes"][SAMPLE]
    b = np.concatenate([xi[:, k * S:(k + 1) * S].cpu().numpy() for k in SAMPLE], axis=1)
    xo, _, _, fails = wilson.solve_many(L, -1, KAPPA, c5["U"], bx, b, tol=1e-12)
    assert fails == 0
    for i, k in enumerate(SAMPLE):
        xg = x[:, k * S:(k + 1) * S].cpu().numpy()
        for f in range(NF):
            ref = xo[f, i * S:(i + 1) * S]
            assert np.linalg.norm(xg[f] - ref) <= 1e-8 * np.linalg.norm(ref), (k, f)
        for f in (0, NF - 1):
            r = b[f, i * S:(i + 1) * S] - wilson.dirac_box(L, -1, KAPPA, c5["U"], bx[i][:4], bx[i][4:8], xg[f])
            assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(b[f, i * S:(i + 1) * S]), (k, f)
