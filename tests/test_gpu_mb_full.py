"""The global pieces of Section 4 at the size and launch configuration `bench.py --workload global` times
(48^4 lattice, 1296 tiles of 8^4 with 4^4 active boxes, kappa 0.12, links exp(0.2 i H), 4 fields at the
u_k of N = 8, c = 0.5), checked through properties that hold at any size (the oracle's W_z needs a
solve on the whole inactive region, out of its reach at 48^4; its element-by-element parity is
test_gpu_mb_w.py's, up to 16^4):

* the generated chi vanishes off dPi, and its support is exactly dPi (dPi_1 from the domain's list
  plus the 1296 * (4^4 - 2^4) sites of dLambda_0);
* W_u chi, applied by a separate call, gives back eta on dPi to the generation's tolerance;
* W_z is affine in z: W_u chi - W_0 chi = u chi (the block and inactive-region solves do not see z);
* the global rest S^r_MB of each field (one inactive-region solve) equals |W_u chi|^2 summed over
  dPi_1 from the applied W;
* sampled rows against the oracle: on dLambda_0 of two blocks (the one at the origin, whose exterior
  shell crosses the antiperiodic time edge, and one inside the lattice) W_u chi is u chi plus the
  block solve of the hops of chi from dPi into the block, computed by the oracle's exterior_source
  and block solver from the same chi and links, element by element.  For one block the sites of dPi
  on its exterior shell are the same as with all blocks (the active boxes' faces lie on the same
  hyperplanes in every tile, and the shell's own perpendicular coordinate is on none of them).
Norms are taken on the device (each field is 2 GB)."""
import numpy as np
import pytest

import synth
from oracle import geometry, mb, wilson

pytestmark = pytest.mark.gpu

L = (48, 48, 48, 48)
KAPPA = 0.12
NF = 4


def test_global_pieces_at_48x4():
    import torch

    from paper_2211_06902_amd import dd

    ctx = dd.Context(0)
    blk = ctx.make_blocks(L, -1, [[8] * 6] * 4, inner_d=2)
    D = ctx.make_inactive(blk)
    U = synth.gauge_field_device(L, 0.2, 7001)
    g = ctx.load_gauge(blk, U, "f32")
    gd = ctx.load_gauge(D, U, "f32")
    Uh = U.cpu().numpy()
    del U
    V = int(np.prod(L))
    eta = synth.spinor_field_device(NF, V, 7002) / np.sqrt(2)
    u = dd.mb_roots(2 * NF, 0.5)
    prm = dd.solve_params(tol=1e-12)

    chi, its, rel, info, st = ctx.mb_generate(blk, g, D, gd, KAPPA, u, eta, tol=1e-10, maxit=60, params=prm)
    assert st == dd.DD_OK and np.all(its > 0) and np.all(rel <= 1e-9), (its, rel)

    # support of chi = dPi
    dpi1 = torch.from_numpy(D.dpi1()).cuda()
    mask = (chi != 0).flatten(2).any(dim=2)  # [NF, V]
    assert bool((mask == mask[0]).all())
    m = mask[0]
    n_dl0 = 1296 * (4**4 - 2**4)
    assert int(m.sum()) == dpi1.numel() + n_dl0 and bool(m[dpi1].all())

    # W_u chi = eta on dPi
    W, info_w, st_w = ctx.mb_apply_W(blk, g, D, gd, KAPPA, u, chi, params=prm)
    assert st_w == dd.DD_OK
    mf = m[None, :, None, None]
    for k in range(NF):
        e = torch.where(mf[0], eta[k], 0)
        res = float(torch.linalg.vector_norm(W[k] - e) / torch.linalg.vector_norm(e))
        assert res <= 1e-9, (k, res)
        assert bool((W[k][~m] == 0).all())

    # sampled dLambda_0 rows against the oracle (field 0)
    bx = blk.tables()[0]
    chi0 = chi[0].cpu().numpy()[None]
    for a in (0, 777):
        box, inn = bx[a:a + 1, :8], bx[a:a + 1, 8:16]
        xi = mb.exterior_source(L, -1, KAPPA, Uh, box, inn, chi0, "all")
        y, _, _, fails = wilson.solve_many(L, -1, KAPPA, Uh, box, xi, tol=1e-13)
        assert fails == 0
        bl = mb.boundary_lists(L, box, inn)[0]
        sites = geometry.box_sites(L, box[0, :4], box[0, 4:8])[bl]
        ref = complex(u[0]) * chi0[0][sites] + y[0, bl]
        got = W[0][torch.from_numpy(sites).cuda()].cpu().numpy()
        assert np.abs(got - ref).max() <= 1e-9 * np.abs(ref).max(), a
    del Uh, chi0

    # W_u chi - W_0 chi = u chi
    W0, _, st0 = ctx.mb_apply_W(blk, g, D, gd, KAPPA, [0.0] * NF, chi, params=prm)
    assert st0 == dd.DD_OK
    for k in range(NF):
        d = W[k] - W0[k] - complex(u[k]) * chi[k]
        assert float(d.abs().max()) <= 1e-12 * float(W[k].abs().max()), k
    del W0

    # S^r_MB per field = |W_u chi|^2 over dPi_1
    Sr, tot, info_s, st_s = ctx.mb_global_action(D, gd, KAPPA, u, chi, params=prm)
    assert st_s == dd.DD_OK
    for k in range(NF):
        ref = float((W[k][dpi1].abs() ** 2).sum())
        assert abs(Sr[k] - ref) <= 1e-9 * ref, (k, Sr[k], ref)
    assert abs(tot - Sr.sum()) <= 1e-12 * abs(tot)
    for h in (gd, g, D, blk):
        h.close()
    ctx.close()
