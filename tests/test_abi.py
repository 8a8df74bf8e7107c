"""CPU checks of the C ABI: the library loads, exports every declared symbol,
and its host geometry tables agree bit for bit with the oracle's geometry."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import geometry
from tests import _cfg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    txt = open(os.path.join(ROOT, "include", "dd.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dd_[a-z_A-Z0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    from paper_2211_06902_amd import dd

    lib = ctypes.CDLL(dd.LIB_PATH)
    syms = _declared_symbols()
    assert len(syms) >= 20
    missing = [s for s in syms if not hasattr(lib, s)]
    assert not missing, missing
    assert dd.version().startswith("libdd")


def _check_tables(blk, L, boxes, inner=None):
    bx, sites, eo, bnd = blk.tables()
    assert blk.n_blocks == len(boxes)
    assert np.array_equal(bx[:, :8], np.asarray(boxes, dtype=np.int32).reshape(-1, 8))
    exp_sites = _cfg.block_sites(L, boxes)
    assert np.array_equal(sites, exp_sites)
    off = _cfg.site_offsets(boxes)
    for k, b in enumerate(boxes):
        _, pos = geometry.box_eo_order(L, b[:4], b[4:8])
        assert np.array_equal(eo[off[k]:off[k + 1]], pos)
    if inner is not None:
        exp = np.concatenate([geometry.inner_boundary_local(L, b, i[:4], i[4:8]) for b, i in zip(boxes, inner)])
        assert np.array_equal(bnd, exp)
        assert np.array_equal(bx[:, 8:16], np.asarray(inner, dtype=np.int32).reshape(-1, 8))
    # links kept by D_Lambda: every forward hop that stays inside its box
    n_links = 0
    for b in boxes:
        e = np.asarray(b[4:8])
        for mu in range(4):
            if e[mu] == L[mu]:
                n_links += int(np.prod(e))
            else:
                n_links += int(np.prod(e)) // e[mu] * (e[mu] - 1)
    assert blk.inner_links == n_links


def test_tiles_c1_both_tilings():
    from paper_2211_06902_amd import dd

    L = _cfg.C1["L"]
    for shift in [(0, 0, 0, 0), (1, 1, 1, 1)]:
        blk = dd.make_blocks(None, L, -1, _cfg.C1["segs"], shift=shift)
        _check_tables(blk, L, geometry.tile_boxes(L, _cfg.C1["segs"], shift=shift))


def test_tiles_c2_and_inner_boundary():
    from paper_2211_06902_amd import dd

    L = (16, 16, 16, 16)
    blk = dd.make_blocks(None, L, -1, [[8, 8]] * 4, inner_d=1)
    boxes = geometry.tile_boxes(L, [[8, 8]] * 4)
    inner = [[1, 1, 1, 1, 6, 6, 6, 6]] * len(boxes)
    _check_tables(blk, L, boxes, inner)
    assert blk.total_bnd_sites == len(boxes) * (6**4 - 4**4)


def test_tiles_c3_uneven():
    from paper_2211_06902_amd import dd

    L = (40, 8, 8, 16)
    segs = [[12, 8, 12, 8], [8], [4, 4], [8, 8]]
    blk = dd.make_blocks(None, L, -1, segs)
    _check_tables(blk, L, geometry.tile_boxes(L, segs))


def test_paper_mode_framed_blocks():
    from paper_2211_06902_amd import dd

    L = (6, 6, 6, 4)
    bd = [2, 1, 2, 1, 2, 1, 0, 0]
    blk = dd.make_blocks_paper(None, L, -1, bd)
    P = geometry.PaperDomains(L, [(2, 1), (2, 1), (2, 1), None])
    boxes = [list(b["omega"][0]) + list(b["omega"][1]) for b in P.blocks]
    inner = [[1, 1, 1, 0, 2, 2, 2, 4]] * len(boxes)
    _check_tables(blk, L, boxes, inner)
    # dLambda_0 from the tables equals the oracle's dLambda_0^a
    _, sites, _, bnd = blk.tables()
    off = _cfg.site_offsets(boxes)
    boff = 0
    for a in range(len(boxes)):
        n = int(P.dlam0_a[a].sum())
        got = sites[off[a] + bnd[boff:boff + n]]
        assert np.array_equal(np.sort(got), np.nonzero(P.dlam0_a[a])[0])
        boff += n


def test_explicit_boxes_wrapping_and_full_span():
    from paper_2211_06902_amd import dd

    L = (4, 4, 2, 2)
    boxes = [[3, 1, 0, 1, 2, 2, 2, 2], [1, 0, 0, 0, 4, 2, 2, 2], [2, 3, 1, 0, 2, 2, 2, 2]]
    blk = dd.make_blocks_boxes(None, L, -1, boxes)
    _check_tables(blk, L, boxes)


@pytest.mark.parametrize("bad", [
    dict(L=(4, 4, 4, 4), segs=[[3, 1], [2, 2], [2, 2], [2, 2]]),   # odd extent
    dict(L=(4, 4, 4, 4), segs=[[2, 2], [2, 2], [2, 2], [2, 4]]),   # does not sum to L
    dict(L=(5, 4, 4, 4), segs=[[5], [2, 2], [2, 2], [2, 2]]),      # odd lattice
])
def test_invalid_geometry_rejected(bad):
    from paper_2211_06902_amd import dd

    with pytest.raises(dd.DDError) as ei:
        dd.make_blocks(None, bad["L"], -1, bad["segs"])
    assert ei.value.status == dd.DD_EINVAL


def test_header_cites_paper_sections():
    txt = open(os.path.join(ROOT, "include", "dd.h")).read()
    for s in ["Section 2", "Section 3", "Section 4", "eq. (localMB)"]:
        assert s in txt


def test_mb_roots_match_the_oracle():
    """The library's host formula for the field parameters u_k against the oracle's roots."""
    import numpy as np

    from oracle import roots
    from paper_2211_06902_amd import dd

    for N, c in [(24, 0.5), (8, 0.3), (2, 0.9)]:
        u = dd.mb_roots(N, c)
        assert u.shape == (N // 2,)
        assert np.max(np.abs(u - roots.mb_roots(N, c)[:N // 2])) <= 1e-15
    for N, c in [(7, 0.5), (8, 1.0), (8, 0.0)]:
        with pytest.raises(dd.DDError):
            dd.mb_roots(N, c)


def test_binding_constants_match_the_header():
    """Every DD_TUNE_* and DD_KCLASS_* value of include/dd.h has the same value in the binding."""
    from paper_2211_06902_amd import dd

    txt = open(os.path.join(ROOT, "include", "dd.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    found = re.findall(r"\bDD_((?:TUNE|KCLASS)_[A-Z0-9_]+)\s*=\s*(\d+)", txt)
    assert len(found) >= 15
    for name, val in found:
        if name == "KCLASS_COUNT":
            continue
        assert getattr(dd, name) == int(val), name


def test_solve_params_defaults():
    """The header's documented defaults: tolerance 1e-10, library inner tolerance, polls every 2
    BiCGStab iterations (host-only call, no device needed)."""
    from paper_2211_06902_amd import dd

    p = dd.solve_params()
    assert p.tol == 1e-10
    assert p.inner_tol <= 0
    assert p.check_every == 2
    assert p.restart == 16


def _oracle_exterior_hops(L, boxes, inner, tbc=-1):
    """(block, box-local site, code, exterior site) of every hop into a box from a dPi site outside it,
    from the oracle's sets (geometry.BoxDomains); code as in dd_blocks_exterior."""
    B = geometry.BoxDomains(L, boxes, inner)
    out = set()
    for k, bx in enumerate(np.asarray(boxes).reshape(-1, 8)):
        e = bx[4:8]
        y = np.indices(e).reshape(4, -1).T
        x = (y + bx[:4]) % np.asarray(L)
        for mu in range(4):
            if e[mu] == L[mu]:
                continue
            for f, step in enumerate((1, -1)):
                yy = y[:, mu] + step
                leave = (yy < 0) | (yy >= e[mu])
                xn = x.copy()
                xn[:, mu] = (xn[:, mu] + step) % L[mu]
                n = ((xn[:, 0] * L[1] + xn[:, 1]) * L[2] + xn[:, 2]) * L[3] + xn[:, 3]
                for s in np.nonzero(leave)[0]:
                    part = 1 if B.dPi1[n[s]] else (2 if B.dlam0[n[s]] else 0)
                    if not part:
                        continue
                    sign = tbc < 0 and mu == 0 and ((f == 0 and x[s, 0] == L[0] - 1) or (f == 1 and x[s, 0] == 0))
                    out.add((k, int(s), (2 * mu + f) | (8 if sign else 0) | (part << 4), int(n[s])))
    return out


@pytest.mark.parametrize("case", ["paper_3d", "paper_4d_wrap", "tiles_inner"])
def test_exterior_hops_match_oracle(case):
    """The hop list of the multi-boson exterior source is bit-exact against the oracle's sets."""
    from paper_2211_06902_amd import dd

    if case == "paper_3d":
        L, bd = (6, 6, 6, 4), [2, 1, 2, 1, 2, 1, 0, 0]
        blk = dd.make_blocks_paper(None, L, -1, bd)
    elif case == "paper_4d_wrap":
        L, bd = (12, 12, 12, 12), [4, 2] * 4
        blk = dd.make_blocks_paper(None, L, -1, bd)
    else:
        L = (8, 8, 8, 8)
        blk = dd.make_blocks(None, L, -1, [[4, 4]] * 4, inner_d=1)
    bx = blk.tables()[0]
    b, s, c, n = blk.exterior()
    got = set(zip(b.tolist(), s.tolist(), c.tolist(), n.tolist()))
    assert len(got) == len(b)
    exp = _oracle_exterior_hops(L, bx[:, :8], bx[:, 8:16])
    assert got == exp
    assert len(exp) > 0
    # grouped by block and site, in increasing order
    key = b.astype(np.int64) * (1 << 32) + s
    assert np.all(np.diff(key) >= 0)
    if case.startswith("paper"):
        # the exterior boundary of a framed block lies on dPi: every exterior hop is listed
        for k in range(blk.n_blocks):
            e = bx[k, 4:8]
            n_ext = sum(int(np.prod(e)) // e[m] * 2 for m in range(4) if e[m] < L[m])
            assert np.sum(b == k) == n_ext


@pytest.mark.parametrize("case", ["paper_3d", "paper_4d"])
def test_frame_tables(case):
    """Frames (box minus inner box): same boxes and layout as their blocks, no dLambda_0 sites, no
    exterior hops, and exactly the links with both ends in the frame kept."""
    from paper_2211_06902_amd import dd

    if case == "paper_3d":
        L, bd = (6, 6, 6, 4), [2, 1, 2, 1, 2, 1, 0, 0]
    else:
        L, bd = (12, 12, 12, 12), [4, 2] * 4
    blk = dd.make_blocks_paper(None, L, -1, bd)
    fr = dd.make_frames(None, blk)
    bx, sites, eo, _ = blk.tables()
    fbx, fsites, feo, _ = fr.tables()
    assert np.array_equal(bx, fbx) and np.array_equal(sites, fsites) and np.array_equal(eo, feo)
    assert fr.total_sites == blk.total_sites and fr.total_bnd_sites == 0
    assert len(fr.exterior()[0]) == 0
    links = 0
    for b in bx:
        e = b[4:8]
        m = np.zeros(tuple(e), dtype=bool)
        m[...] = True
        ho, he = b[8:12], b[12:16]
        m[ho[0]:ho[0] + he[0], ho[1]:ho[1] + he[1], ho[2]:ho[2] + he[2], ho[3]:ho[3] + he[3]] = False
        for mu in range(4):
            if e[mu] == L[mu]:
                links += int(np.sum(m & np.roll(m, -1, axis=mu)))
            else:
                sl = [slice(None)] * 4
                sl2 = [slice(None)] * 4
                sl[mu] = slice(0, e[mu] - 1)
                sl2[mu] = slice(1, e[mu])
                links += int(np.sum(m[tuple(sl)] & m[tuple(sl2)]))
    assert fr.inner_links == links
    with pytest.raises(dd.DDError):
        dd.make_frames(None, dd.make_blocks(None, (8, 8, 8, 8), -1, [[4, 4]] * 4))


@pytest.mark.parametrize("case", ["tiles_inner", "paper_3d"])
def test_inactive_domain_tables(case):
    """The inactive-region domain (dd_make_inactive): one block spanning the lattice; its dPi_1 list is
    the oracle's set; its exterior hops are exactly the hops from the active boxes into Lambda_1 (part
    dLambda_0, antiperiodic sign on the time edge); it keeps exactly the links with both ends in
    Lambda_1."""
    from oracle import geometry
    from paper_2211_06902_amd import dd

    if case == "paper_3d":
        L, bd = (6, 6, 6, 4), [2, 1, 2, 1, 2, 1, 0, 0]
        blk = dd.make_blocks_paper(None, L, -1, bd)
    else:
        L = (8, 8, 8, 8)
        blk = dd.make_blocks(None, L, -1, [[4, 4]] * 4, inner_d=1)
    bx = blk.tables()[0]
    D = dd.make_inactive(None, blk)
    V = int(np.prod(L))
    assert D.n_blocks == 1 and D.total_sites == V
    dbx = D.tables()[0][0]
    assert list(dbx[:4]) == [0, 0, 0, 0] and list(dbx[4:8]) == list(L)
    P = geometry.BoxDomains(L, bx[:, :8], bx[:, 8:16])
    assert np.array_equal(D.dpi1(), np.nonzero(P.dPi1)[0])
    nb = geometry.neighbours(L)
    x0 = geometry.coords(L)[:, 0]
    exp = set()
    for n in np.nonzero(P.lam1)[0]:
        for mu in range(4):
            for f in range(2):
                m = nb[n, 2 * mu + f]
                if P.lam0[m]:
                    sign = mu == 0 and ((f == 0 and x0[n] == L[0] - 1) or (f == 1 and x0[n] == 0))
                    exp.add((0, int(n), (2 * mu + f) | (8 if sign else 0) | (2 << 4), int(m)))
    b, s, c, nbr = D.exterior()
    got = set(zip(b.tolist(), s.tolist(), c.tolist(), nbr.tolist()))
    assert len(got) == len(b) and got == exp and len(exp) > 0
    links = sum(1 for n in np.nonzero(P.lam1)[0] for mu in range(4) if P.lam1[nb[n, 2 * mu]])
    assert D.inner_links == links
    D.close()
    blk.close()


def test_block_size_limit_of_32bit_offsets():
    """A block whose FP64 links would reach 4 GiB is refused (the kernels address a block's buffers with
    32-bit byte offsets): the inactive region of 64^4 is one such block; 48^4 is accepted."""
    from paper_2211_06902_amd import dd

    blk = dd.make_blocks(None, (64, 64, 64, 64), -1, [[8] * 8] * 4, inner_d=1)
    with pytest.raises(dd.DDError):
        dd.make_inactive(None, blk)
    blk.close()
    blk = dd.make_blocks(None, (48, 48, 48, 48), -1, [[8] * 6] * 4, inner_d=1)
    D = dd.make_inactive(None, blk)
    assert D.total_sites == 48**4 and D.total_sites * 48 * 8 < 2**32
    D.close()
    blk.close()


def test_null_arguments_are_refused_without_a_device():
    """Every entry point of the global pieces, the BiCGStab autotuner and the inactive-region builder
    checks its handles before it touches a device: all-null calls return DD_EINVAL (no GPU here)."""
    import ctypes

    from paper_2211_06902_amd import dd

    L = dd._lib
    N = None
    assert L.dd_mb_global_action(N, N, N, 0.1, 1, N, N, N, N, N, N) == dd.DD_EINVAL
    assert L.dd_mb_apply_W(N, N, N, N, N, 0.1, 1, N, N, N, N, N) == dd.DD_EINVAL
    assert L.dd_mb_generate(N, N, N, N, N, 0.1, 1, N, N, N, 1e-10, 10, N, N, N, N) == dd.DD_EINVAL
    assert L.dd_mb_log_reweight(N, N, N, N, N, 0.1, 2, 0.5, 1, 1, N, N, N, N, N) == dd.DD_EINVAL
    assert L.dd_autotune_bicgstab(N, N, N, 0.1, N, N, 1, N, N, N, 0, N, N) == dd.DD_EINVAL
    out = ctypes.c_void_p()
    assert L.dd_make_inactive(N, N, ctypes.byref(out)) == dd.DD_EINVAL
    assert L.dd_make_inactive(N, N, N) == dd.DD_EINVAL
