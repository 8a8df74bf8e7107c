// Block geometry of libdd (host): boxes, shapes, even-odd permutations,
// neighbour tables and dLambda_0 lists.
//
// Paper Section 2: blocks Lambda_0^a are hyperrectangles; the solve domains
// are boxes (tiles, or the framed blocks Omega_0^a = Lambda_0^a u Phi_1^a);
// dLambda_0^a holds the sites of the active box with a neighbour outside it.
// Section 3: D_X drops the hops from outside X (Dirichlet restriction), which
// the neighbour tables encode as -1 entries.
#include <algorithm>
#include <cstring>
#include <map>
#include <tuple>

#include "dd_geometry.h"

namespace dd {

namespace {

struct ShapeKey {
    int e[4], full[4], opar, tw, hole, hio[4], hie[4];
    bool operator<(const ShapeKey &o) const
    {
        return std::tie(e[0], e[1], e[2], e[3], full[0], full[1], full[2], full[3], opar, tw, hole, hio[0], hio[1],
                        hio[2], hio[3], hie[0], hie[1], hie[2], hie[3]) <
               std::tie(o.e[0], o.e[1], o.e[2], o.e[3], o.full[0], o.full[1], o.full[2], o.full[3], o.opar, o.tw,
                        o.hole, o.hio[0], o.hio[1], o.hio[2], o.hio[3], o.hie[0], o.hie[1], o.hie[2], o.hie[3]);
    }
};

inline int lidx(const int e[4], const int y[4]);

inline bool in_hole(const Shape &sh, const int y[4])
{
    if (!sh.hole) return false;
    if (sh.hole == 2) return sh.mask[lidx(sh.e, y)] != 0;
    for (int m = 0; m < 4; m++)
        if (y[m] < sh.hio[m] || y[m] >= sh.hio[m] + sh.hie[m]) return false;
    return true;
}

inline int lidx(const int e[4], const int y[4]) { return ((y[0] * e[1] + y[1]) * e[2] + y[2]) * e[3] + y[3]; }

inline void lcoords(const int e[4], int s, int y[4])
{
    y[3] = s % e[3];
    s /= e[3];
    y[2] = s % e[2];
    s /= e[2];
    y[1] = s % e[1];
    s /= e[1];
    y[0] = s;
}

// Sites per parity of an x0-slice if the hop's x0-walk applies to the shape,
// else 0: checked on the finished table, entry by entry.  A slice holds
// e1*e2*e3 (even) sites, half of each parity, and the eo order inside a slice
// is the canonical one, so away from the slice ends the x0-neighbour of eo
// site h sits at h +/- hs of the other parity.
int walk_slice(const Shape &sh, const int32_t *tab)
{
    const int hs = sh.e[1] * sh.e[2] * sh.e[3] / 2;
    if (sh.full[0] || hs > kTile || hs * sh.e[0] != sh.h) return 0;
    for (int slot = 0; slot < sh.S; slot++) {
        const int h = slot % sh.h, q = h / hs;
        const int32_t *t = tab + (size_t)slot * 8;
        const int32_t up = q + 1 < sh.e[0] ? h + hs : -1, dn = q > 0 ? h - hs : -1;
        // a dropped hop (Dirichlet face, or a frame's hole) is always fine
        if ((t[0] >= 0 && (t[0] & kNbrMask) != up) || (t[1] >= 0 && (t[1] & kNbrMask) != dn)) return 0;
        if ((up < 0 && t[0] >= 0) || (dn < 0 && t[1] >= 0)) return 0;
        for (int k = 2; k < 8; k++)
            if (t[k] >= 0 && (t[k] & kNbrMask) / hs != q) return 0;
    }
    return hs;
}

// Build the permutation and neighbour table of one shape; returns links kept.
int64_t build_shape(Shape &sh, int tbc, std::vector<int32_t> &perm, std::vector<int32_t> &nbr)
{
    const int *e = sh.e;
    sh.S = e[0] * e[1] * e[2] * e[3];
    sh.h = sh.S / 2;
    sh.perm_off = (int64_t)perm.size();
    sh.nbr_off = (int64_t)nbr.size();
    std::vector<int32_t> pos(sh.S);
    int ne = 0, no = 0;
    for (int p = 0; p < 2; p++)
        for (int s = 0; s < sh.S; s++) {
            int y[4];
            lcoords(e, s, y);
            const int par = (sh.opar + y[0] + y[1] + y[2] + y[3]) & 1;
            if (par != p) continue;
            pos[s] = p == 0 ? ne : sh.h + no;
            (p == 0 ? ne : no)++;
            perm.push_back(s);
        }
    nbr.resize(nbr.size() + (size_t)sh.S * 8);
    int32_t *tab = nbr.data() + sh.nbr_off;
    int64_t links = 0;
    for (int slot = 0; slot < sh.S; slot++) {
        const int p = slot >= sh.h;
        int y[4];
        lcoords(e, perm[sh.perm_off + slot], y);
        const bool hole_site = in_hole(sh, y);
        for (int mu = 0; mu < 4; mu++) {
            for (int f = 0; f < 2; f++) {
                int yy[4] = {y[0], y[1], y[2], y[3]};
                bool in = true;
                int link_origin;  // local mu-coordinate of the link's lower end
                if (f == 0) {
                    link_origin = y[mu];
                    yy[mu] = y[mu] + 1;
                    if (yy[mu] == e[mu]) {
                        if (sh.full[mu]) yy[mu] = 0;
                        else in = false;
                    }
                } else {
                    yy[mu] = y[mu] - 1;
                    if (yy[mu] < 0) {
                        if (sh.full[mu]) yy[mu] = e[mu] - 1;
                        else in = false;
                    }
                    link_origin = yy[mu];
                }
                int32_t entry = -1;
                if (in && (hole_site || in_hole(sh, yy))) in = false;
                if (in) {
                    entry = pos[lidx(e, yy)] - (1 - p) * sh.h;
                    if (tbc < 0 && mu == 0 && link_origin == sh.tw) entry |= kNbrSign;
                    if (f == 0) links++;
                }
                tab[(size_t)slot * 8 + 2 * mu + f] = entry;
            }
        }
    }
    sh.walk_hs = walk_slice(sh, tab);
    return links;
}

// Exterior hops of the multi-boson source (Section 4, eq. localMB): the
// hyperplanes dPi are the sites with some coordinate on a face coordinate
// (first or last) of an inner box, in the directions where that box does not
// span the lattice; the sets dLambda_0 (boundary sites of the inner boxes)
// and dPi_1 (dPi outside the inner boxes) are its two parts.  For every
// block, the hops into the box from exterior sites in either part are listed,
// grouped by receiving site.  Nothing is built when every inner box is its
// block (no frames).
// The active sets on the lattice (global canonical index): lam0 (the union
// of the inner boxes), dlam0 (their boundary sites: a coordinate on a face of
// the box in a direction where it does not span the lattice), and face[m]
// (the coordinates along m that carry a face of some inner box: dPi is the
// sites with some coordinate among them).
void active_sets(const dd_blocks *B, std::vector<uint8_t> &lam0, std::vector<uint8_t> &dlam0,
                 std::vector<uint8_t> (&face)[4])
{
    const int *L = B->L;
    const int64_t V = (int64_t)L[0] * L[1] * L[2] * L[3];
    auto gidx = [&](const int x[4]) { return (((int64_t)x[0] * L[1] + x[1]) * L[2] + x[2]) * L[3] + x[3]; };
    lam0.assign(V, 0);
    dlam0.assign(V, 0);
    for (int m = 0; m < 4; m++) face[m].assign(L[m], 0);
    for (int k = 0; k < B->nb; k++) {
        const int32_t *r = &B->box[16 * k];
        int io[4], ie[4];
        for (int m = 0; m < 4; m++) {
            io[m] = (r[m] + r[8 + m]) % L[m];
            ie[m] = r[12 + m];
            if (ie[m] < L[m]) {
                face[m][io[m]] = 1;
                face[m][(io[m] + ie[m] - 1) % L[m]] = 1;
            }
        }
        const int S = ie[0] * ie[1] * ie[2] * ie[3];
        for (int q = 0; q < S; q++) {
            int y[4], x[4];
            lcoords(ie, q, y);
            bool bnd = false;
            for (int m = 0; m < 4; m++) {
                x[m] = (io[m] + y[m]) % L[m];
                if (ie[m] < L[m] && (y[m] == 0 || y[m] == ie[m] - 1)) bnd = true;
            }
            lam0[gidx(x)] = 1;
            if (bnd) dlam0[gidx(x)] = 1;
        }
    }
}

void build_exterior(dd_blocks *B)
{
    const int *L = B->L;
    bool framed = false;
    for (int k = 0; k < B->nb; k++)
        for (int m = 0; m < 4; m++) framed = framed || B->box[16 * k + 12 + m] != B->box[16 * k + 4 + m];
    if (!framed || B->hole[0]) return;  // no frames, or frame domains themselves
    auto gidx = [&](const int x[4]) { return (((int64_t)x[0] * L[1] + x[1]) * L[2] + x[2]) * L[3] + x[3]; };
    std::vector<uint8_t> face[4], lam0, dlam0;
    active_sets(B, lam0, dlam0, face);
    B->xg_first.assign(1, 0);
    for (int k = 0; k < B->nb; k++) {
        const int32_t *r = &B->box[16 * k];
        const int o[4] = {r[0], r[1], r[2], r[3]}, e[4] = {r[4], r[5], r[6], r[7]};
        const int S = e[0] * e[1] * e[2] * e[3];
        for (int s = 0; s < S; s++) {
            int y[4], x[4];
            lcoords(e, s, y);
            bool shell = false;
            for (int m = 0; m < 4; m++) {
                x[m] = (o[m] + y[m]) % L[m];
                if (e[m] < L[m] && (y[m] == 0 || y[m] == e[m] - 1)) shell = true;
            }
            if (!shell) continue;
            const size_t first = B->x_code.size();
            for (int mu = 0; mu < 4; mu++) {
                if (e[mu] == L[mu]) continue;  // the box wraps onto itself along mu
                for (int f = 0; f < 2; f++) {
                    const int yy = y[mu] + (f ? -1 : 1);
                    if (yy >= 0 && yy < e[mu]) continue;
                    int xn[4] = {x[0], x[1], x[2], x[3]};
                    xn[mu] = (x[mu] + (f ? L[mu] - 1 : 1)) % L[mu];
                    const int64_t n = gidx(xn);
                    bool on_pi = false;
                    for (int m = 0; m < 4; m++) on_pi = on_pi || face[m][xn[m]];
                    if (!on_pi) continue;
                    const int part = lam0[n] ? (dlam0[n] ? 2 : 0) : 1;
                    if (!part) continue;
                    const bool sign = B->tbc < 0 && mu == 0 &&
                                      ((f == 0 && x[0] == L[0] - 1) || (f == 1 && x[0] == 0));
                    B->x_code.push_back((2 * mu + f) | (sign ? 8 : 0) | (part << 4));
                    B->x_nbr.push_back(n);
                    B->x_link.push_back(4 * (f ? n : gidx(x)) + mu);
                }
            }
            if (B->x_code.size() > first) {
                B->xg_block.push_back(k);
                B->xg_site.push_back(s);
                B->xg_first.push_back((int32_t)B->x_code.size());
            }
        }
    }
}

}  // namespace

std::string build_geometry(dd_blocks *B, const int L[4], int tbc, int n, const int32_t *boxes,
                           const int32_t *inner, bool frames)
{
    for (int m = 0; m < 4; m++)
        if (L[m] < 2 || (L[m] & 1)) return "lattice extents must be even and >= 2";
    if (tbc != 1 && tbc != -1) return "time_bc must be +1 (periodic) or -1 (antiperiodic)";
    if (n < 0) return "negative block count";
    for (int m = 0; m < 4; m++) B->L[m] = L[m];
    B->tbc = tbc;
    B->nb = n;
    B->box.assign((size_t)n * 16, 0);
    B->soff.assign(n + 1, 0);
    B->boff.assign(n + 1, 0);
    B->shape_of.assign(n, 0);
    B->hole.assign(n, frames ? 1 : 0);
    std::map<ShapeKey, int> shape_ids;
    std::vector<int64_t> shape_links;
    for (int k = 0; k < n; k++) {
        const int32_t *bx = boxes + 8 * k;
        int o[4], e[4], io[4], ie[4];
        for (int m = 0; m < 4; m++) {
            o[m] = ((bx[m] % L[m]) + L[m]) % L[m];
            e[m] = bx[4 + m];
            if (e[m] < 2 || (e[m] & 1) || e[m] > L[m]) return "block extents must be even, >= 2 and <= L";
            io[m] = inner ? inner[8 * k + m] : 0;
            ie[m] = inner ? inner[8 * k + 4 + m] : e[m];
            if (io[m] < 0 || ie[m] < 1 || io[m] + ie[m] > e[m]) return "inner box must lie inside its block";
        }
        if (frames) {
            bool proper = false;
            for (int m = 0; m < 4; m++) proper = proper || ie[m] != e[m];
            if (!proper) return "a frame needs an inner box smaller than its block";
        }
        ShapeKey key;
        for (int m = 0; m < 4; m++) {
            key.e[m] = e[m];
            key.full[m] = e[m] == L[m];
        }
        key.opar = (o[0] + o[1] + o[2] + o[3]) & 1;
        key.hole = frames ? 1 : 0;
        for (int m = 0; m < 4; m++) {
            key.hio[m] = frames ? io[m] : 0;
            key.hie[m] = frames ? ie[m] : 0;
        }
        key.tw = -1;
        if (tbc < 0) {
            const int tw = ((L[0] - 1 - o[0]) % L[0] + L[0]) % L[0];
            if (key.full[0] || tw <= e[0] - 2) key.tw = tw;
        }
        auto it = shape_ids.find(key);
        int sid;
        if (it == shape_ids.end()) {
            Shape sh;
            std::memcpy(sh.e, key.e, sizeof(sh.e));
            std::memcpy(sh.full, key.full, sizeof(sh.full));
            sh.opar = key.opar;
            sh.tw = key.tw;
            sh.hole = key.hole;
            std::memcpy(sh.hio, key.hio, sizeof(sh.hio));
            std::memcpy(sh.hie, key.hie, sizeof(sh.hie));
            const int64_t links = build_shape(sh, tbc, B->perm, B->nbr);
            sh.links = links;
            sid = (int)B->shapes.size();
            B->shapes.push_back(sh);
            shape_links.push_back(links);
            shape_ids[key] = sid;
        } else {
            sid = it->second;
        }
        B->shape_of[k] = sid;
        const Shape &sh = B->shapes[sid];
        // the kernels address a block's buffers with 32-bit byte offsets from
        // its base: its FP64 links (4 directions x 6 complex entries) must stay
        // below 4 GiB
        if ((int64_t)sh.S * kLinkReals * 8 >= ((int64_t)1 << 32))
            return "block too large for the kernels' 32-bit offsets (a block holds at most 11184810 sites)";
        B->soff[k + 1] = B->soff[k] + sh.S;
        B->inner_links += shape_links[sid];
        B->max_h = std::max(B->max_h, sh.h);
        int32_t *rec = &B->box[(size_t)16 * k];
        for (int m = 0; m < 4; m++) {
            rec[m] = o[m];
            rec[4 + m] = e[m];
            rec[8 + m] = io[m];
            rec[12 + m] = ie[m];
        }
        // dLambda_0: inner-box sites with a lattice neighbour outside the inner box.
        // Along a direction where the inner box spans the lattice the neighbours wrap inside.
        // (A frame has none: its inner box is not part of its domain.)
        for (int s = 0; s < (frames ? 0 : sh.S); s++) {
            int y[4];
            lcoords(e, s, y);
            bool inside = true, bnd = false;
            for (int m = 0; m < 4; m++) {
                if (y[m] < io[m] || y[m] >= io[m] + ie[m]) inside = false;
                if (ie[m] < L[m] && (y[m] == io[m] || y[m] == io[m] + ie[m] - 1)) bnd = true;
            }
            if (inside && bnd) B->bnd.push_back(s);
        }
        B->boff[k + 1] = (int64_t)B->bnd.size();
    }
    B->walk = n > 0;
    for (const Shape &sh : B->shapes) B->walk = B->walk && sh.walk_hs > 0;
    build_exterior(B);
    return "";
}

std::string build_inactive(dd_blocks *D, const dd_blocks *B)
{
    const int *L = B->L;
    const int64_t V = (int64_t)L[0] * L[1] * L[2] * L[3];
    if (V > ((int64_t)1 << 30)) return "lattice too large for one inactive-region domain";
    auto gidx = [&](const int x[4]) { return (((int64_t)x[0] * L[1] + x[1]) * L[2] + x[2]) * L[3] + x[3]; };
    std::vector<uint8_t> face[4], lam0, dlam0;
    active_sets(B, lam0, dlam0, face);
    int64_t n_in = 0;
    for (int64_t n = 0; n < V; n++) n_in += lam0[n] == 0;
    if (n_in == 0) return "the active boxes cover the lattice: no inactive region";
    const int32_t box[8] = {0, 0, 0, 0, L[0], L[1], L[2], L[3]};
    const std::string msg = build_geometry(D, L, B->tbc, 1, box, box, false);
    if (!msg.empty()) return msg;
    // the active boxes become the shape's excluded sites (its local canonical
    // index is the global one: origin 0, extent L)
    Shape &sh = D->shapes[0];
    sh.hole = 2;
    sh.mask = lam0;
    D->perm.clear();
    D->nbr.clear();
    sh.links = build_shape(sh, B->tbc, D->perm, D->nbr);
    D->inner_links = sh.links;
    D->walk = sh.walk_hs > 0;
    D->hole.assign(1, 2);
    D->inactive = true;
    // hops from the active boxes into the domain, grouped by receiving site
    D->xg_block.clear();
    D->xg_site.clear();
    D->x_code.clear();
    D->x_nbr.clear();
    D->x_link.clear();
    D->xg_first.assign(1, 0);
    D->dpi1.clear();
    for (int64_t n = 0; n < V; n++) {
        if (lam0[n]) continue;
        int x[4];
        {
            int64_t t = n;
            x[3] = (int)(t % L[3]);
            t /= L[3];
            x[2] = (int)(t % L[2]);
            t /= L[2];
            x[1] = (int)(t % L[1]);
            x[0] = (int)(t / L[1]);
        }
        bool on_pi = false;
        for (int m = 0; m < 4; m++) on_pi = on_pi || face[m][x[m]];
        if (on_pi) D->dpi1.push_back(n);
        const size_t first = D->x_code.size();
        for (int mu = 0; mu < 4; mu++)
            for (int f = 0; f < 2; f++) {
                int xn[4] = {x[0], x[1], x[2], x[3]};
                xn[mu] = (x[mu] + (f ? L[mu] - 1 : 1)) % L[mu];
                const int64_t nn = gidx(xn);
                if (!lam0[nn]) continue;
                const bool sign = B->tbc < 0 && mu == 0 && ((f == 0 && x[0] == L[0] - 1) || (f == 1 && x[0] == 0));
                D->x_code.push_back((2 * mu + f) | (sign ? 8 : 0) | (2 << 4));
                D->x_nbr.push_back(nn);
                D->x_link.push_back(4 * (f ? nn : n) + mu);
            }
        if (D->x_code.size() > first) {
            D->xg_block.push_back(0);
            D->xg_site.push_back((int32_t)n);
            D->xg_first.push_back((int32_t)D->x_code.size());
        }
    }
    return "";
}

std::vector<uint8_t> hole_slots(const dd_blocks *B)
{
    bool any = false;
    for (const Shape &sh : B->shapes) any = any || sh.hole != 0;
    if (!any) return {};
    std::vector<uint8_t> out((size_t)B->soff[B->nb], 0);
    for (int b = 0; b < B->nb; b++) {
        const Shape &sh = B->shapes[B->shape_of[b]];
        if (!sh.hole) continue;
        for (int s = 0; s < sh.S; s++) {
            int y[4];
            lcoords(sh.e, B->perm[sh.perm_off + s], y);
            out[(size_t)B->soff[b] + s] = in_hole(sh, y) ? 1 : 0;
        }
    }
    return out;
}

}  // namespace dd
