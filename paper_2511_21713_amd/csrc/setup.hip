// Host-side topology preprocessing: surfaces, adjacency, Morton blocks for the
// regular boundary-element assembly, touching panel pairs and the FEM sliced-ELL
// pattern.  Integer work only; every floating-point quantity of the method is
// computed on the device.
#include <algorithm>
#include <cmath>
#include <map>
#include <numeric>
#include <unordered_map>

#include "pbfb_internal.hpp"

namespace pbfb {

static uint32_t spread10(uint32_t v)
{
    v &= 1023u;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

int tile_shape_index(int ta, int tb)
{
    for (int k = 0; k < N_TILE_SHAPES; ++k)
        if (TILE_SHAPES[k].ta == ta && TILE_SHAPES[k].tb == tb) return k;
    return -1;
}

// Blocks of `bs` consecutive Morton-ordered triangles: their vertex lists
// (ascending operator index), for every local vertex the (triangle-in-block
// * 3 + corner) slots that touch it, and a colouring of the blocks in which
// blocks of one colour share no vertex.
const BlockSide &block_side(SurfaceTopo &S, int bs)
{
    auto found = S.sides.find(bs);
    if (found != S.sides.end()) return found->second;
    BlockSide B;
    B.bs = bs;
    B.nb = (S.nt + bs - 1) / bs;
    B.pref.assign(B.nb + 1, 0);
    B.nvb.assign(B.nb, 0);
    std::vector<std::vector<int32_t>> blk_verts(B.nb); // operator (Morton) indices, ascending
    for (int64_t b = 0; b < B.nb; ++b) {
        std::vector<int32_t> vs;
        for (int k = 0; k < bs; ++k) {
            int64_t m = b * bs + k;
            if (m >= S.nt) break;
            int32_t t = S.morton[m];
            for (int a = 0; a < 3; ++a) vs.push_back(S.minv[S.tri[3 * t + a]]);
        }
        std::sort(vs.begin(), vs.end());
        vs.erase(std::unique(vs.begin(), vs.end()), vs.end());
        blk_verts[b] = vs;
        B.nvb[b] = (int32_t)vs.size();
        B.pref[b + 1] = B.pref[b] + B.nvb[b];
    }
    B.S = B.pref[B.nb];
    B.vid.resize(B.S);
    B.slots.assign(B.S * MAXS, -1);
    std::vector<std::vector<int32_t>> vblocks(S.nv); // blocks of each operator index
    for (int64_t b = 0; b < B.nb; ++b) {
        const auto &vs = blk_verts[b];
        std::copy(vs.begin(), vs.end(), B.vid.begin() + B.pref[b]);
        std::vector<int> fill(vs.size(), 0);
        for (int k = 0; k < bs; ++k) {
            int64_t m = b * bs + k;
            if (m >= S.nt) break;
            int32_t t = S.morton[m];
            for (int a = 0; a < 3; ++a) {
                int32_t v = S.minv[S.tri[3 * t + a]];
                int32_t li = int32_t(std::lower_bound(vs.begin(), vs.end(), v) - vs.begin());
                PB_CHECK(fill[li] < MAXS, PBFB_EMESH,
                         "a surface vertex has more than " + std::to_string(MAXS) + " triangles");
                B.slots[(int64_t(B.pref[b]) + li) * MAXS + fill[li]++] = k * 3 + a;
            }
        }
        for (int32_t v : vs) vblocks[v].push_back(int32_t(b));
        for (int f : fill) B.ms_max = std::max(B.ms_max, f);
    }
    // greedy colouring in block order: the smallest colour no earlier block
    // sharing a vertex with this one has taken
    std::vector<int32_t> color(B.nb, -1);
    std::vector<int64_t> seen;
    for (int64_t b = 0; b < B.nb; ++b) {
        seen.clear();
        for (int32_t v : blk_verts[b])
            for (int32_t o : vblocks[v])
                if (color[o] >= 0) seen.push_back(color[o]);
        std::sort(seen.begin(), seen.end());
        int32_t c = 0;
        for (int64_t x : seen) {
            if (x == c) ++c;
            else if (x > c) break;
        }
        color[b] = c;
        B.ncolor = std::max(B.ncolor, int(c) + 1);
    }
    B.col_ptr.assign(B.ncolor + 1, 0);
    for (int64_t b = 0; b < B.nb; ++b) B.col_ptr[color[b] + 1]++;
    for (int c = 0; c < B.ncolor; ++c) B.col_ptr[c + 1] += B.col_ptr[c];
    B.col_blk.resize(B.nb);
    {
        std::vector<int32_t> fill(B.col_ptr.begin(), B.col_ptr.end() - 1);
        for (int64_t b = 0; b < B.nb; ++b) B.col_blk[fill[color[b]]++] = int32_t(b);
    }
    return S.sides.emplace(bs, std::move(B)).first->second;
}

void build_surface_topo(Problem &p, int which, int64_t ntri, const int32_t *tri)
{
    build_surface_topo_on(p.topo[which], p.nn, p.x.data(), ntri, tri);
}

void build_surface_topo_on(SurfaceTopo &S, int64_t nverts, const double *x, int64_t ntri, const int32_t *tri)
{
    S = SurfaceTopo();
    S.nt = ntri;
    PB_CHECK(ntri >= 4, PBFB_EMESH, "surface needs at least 4 triangles");
    std::vector<int32_t> loc(nverts, -1);
    for (int64_t k = 0; k < 3 * ntri; ++k) {
        PB_CHECK(tri[k] >= 0 && tri[k] < nverts, PBFB_EINVAL, "surface triangle references a node out of range");
        loc[tri[k]] = 0;
    }
    for (int64_t i = 0; i < nverts; ++i)
        if (loc[i] == 0) {
            loc[i] = int32_t(S.g.size());
            S.g.push_back(int32_t(i));
        }
    S.nv = int64_t(S.g.size());
    S.tri.resize(3 * ntri);
    for (int64_t k = 0; k < 3 * ntri; ++k) S.tri[k] = loc[tri[k]];
    // closed oriented 2-manifold: every directed edge once, with its reverse
    {
        std::vector<uint64_t> e;
        e.reserve(3 * ntri);
        for (int64_t t = 0; t < ntri; ++t)
            for (int a = 0; a < 3; ++a) {
                uint32_t i = S.tri[3 * t + a], j = S.tri[3 * t + (a + 1) % 3];
                PB_CHECK(i != j, PBFB_EMESH, "degenerate surface triangle");
                e.push_back((uint64_t(i) << 32) | j);
            }
        std::vector<uint64_t> es = e;
        std::sort(es.begin(), es.end());
        PB_CHECK(std::adjacent_find(es.begin(), es.end()) == es.end(), PBFB_EMESH,
                 "surface has a repeated directed edge (non-manifold or inconsistent orientation)");
        for (uint64_t k : e) {
            uint64_t r = (k << 32) | (k >> 32);
            PB_CHECK(std::binary_search(es.begin(), es.end(), r), PBFB_EMESH, "surface is not closed");
        }
    }
    // vertex -> triangles
    S.v2t_ptr.assign(S.nv + 1, 0);
    for (int64_t k = 0; k < 3 * ntri; ++k) S.v2t_ptr[S.tri[k] + 1]++;
    for (int64_t i = 0; i < S.nv; ++i) S.v2t_ptr[i + 1] += S.v2t_ptr[i];
    S.v2t.resize(3 * ntri);
    {
        std::vector<int32_t> fill(S.v2t_ptr.begin(), S.v2t_ptr.end() - 1);
        for (int64_t t = 0; t < ntri; ++t)
            for (int a = 0; a < 3; ++a) S.v2t[fill[S.tri[3 * t + a]]++] = int32_t(t * 3 + a);
    }
    // Morton order of triangle centroids
    {
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
        for (int64_t i = 0; i < S.nv; ++i)
            for (int d = 0; d < 3; ++d) {
                lo[d] = std::min(lo[d], x[3 * S.g[i] + d]);
                hi[d] = std::max(hi[d], x[3 * S.g[i] + d]);
            }
        double span = std::max({hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2], 1e-30});
        std::vector<std::pair<uint32_t, int32_t>> key(ntri);
        for (int64_t t = 0; t < ntri; ++t) {
            uint32_t code = 0;
            for (int d = 0; d < 3; ++d) {
                double c = 0;
                for (int a = 0; a < 3; ++a) c += x[3 * S.g[S.tri[3 * t + a]] + d];
                c = (c / 3.0 - lo[d]) / span;
                code |= spread10(uint32_t(std::min(1023.0, std::max(0.0, c * 1023.0)))) << d;
            }
            key[t] = {code, int32_t(t)};
        }
        std::sort(key.begin(), key.end());
        S.morton.resize(ntri);
        for (int64_t m = 0; m < ntri; ++m) S.morton[m] = key[m].second;
    }
    // Morton vertex order: first appearance along the Morton triangle order,
    // so that the vertices of a block of consecutive triangles have nearby
    // operator indices
    S.minv.assign(S.nv, -1);
    S.mvert.clear();
    for (int64_t m = 0; m < ntri; ++m)
        for (int a = 0; a < 3; ++a) {
            const int32_t v = S.tri[3 * S.morton[m] + a];
            if (S.minv[v] < 0) {
                S.minv[v] = int32_t(S.mvert.size());
                S.mvert.push_back(v);
            }
        }
    S.gmv.resize(S.nv);
    for (int64_t k = 0; k < S.nv; ++k) S.gmv[k] = S.g[S.mvert[k]];
    // blocks of the default tile shape (other block sizes are built when a
    // shape using them is timed or chosen)
    block_side(S, TILE_SHAPES[0].ta);
    block_side(S, TILE_SHAPES[0].tb);
    // 1-ring of each vertex (itself and every vertex sharing a triangle), ascending
    S.ring_ptr.assign(S.nv + 1, 0);
    S.ring.clear();
    S.max_ring = 0;
    {
        std::vector<int32_t> r;
        for (int64_t i = 0; i < S.nv; ++i) {
            r.assign(1, int32_t(i));
            for (int32_t e = S.v2t_ptr[i]; e < S.v2t_ptr[i + 1]; ++e)
                for (int b = 0; b < 3; ++b) r.push_back(S.tri[3 * (S.v2t[e] / 3) + b]);
            std::sort(r.begin(), r.end());
            r.erase(std::unique(r.begin(), r.end()), r.end());
            PB_CHECK(r.size() <= size_t(MAXRING), PBFB_EMESH, "surface vertex with more than 63 neighbours");
            S.max_ring = std::max(S.max_ring, int(r.size()));
            S.ring.insert(S.ring.end(), r.begin(), r.end());
            S.ring_ptr[i + 1] = int32_t(S.ring.size());
        }
    }
    // touching pairs, grouped by the first triangle
    S.tp_ptr.assign(ntri + 1, 0);
    S.tp_sig.clear();
    std::vector<int32_t> nb;
    for (int64_t t = 0; t < ntri; ++t) {
        nb.clear();
        for (int a = 0; a < 3; ++a) {
            int32_t v = S.tri[3 * t + a];
            for (int32_t e = S.v2t_ptr[v]; e < S.v2t_ptr[v + 1]; ++e) nb.push_back(S.v2t[e] / 3);
        }
        std::sort(nb.begin(), nb.end());
        nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
        S.tp_sig.insert(S.tp_sig.end(), nb.begin(), nb.end());
        S.tp_ptr[t + 1] = int32_t(S.tp_sig.size());
    }
}

void build_fem_topology(Problem &p, std::vector<int32_t> &sptr, std::vector<int32_t> &col,
                        std::vector<int32_t> &n2t_ptr, std::vector<int32_t> &n2t, std::vector<int32_t> &slot4,
                        std::vector<int32_t> &diag, std::vector<int32_t> cslot[2])
{
    const int64_t nn = p.nn, nt = p.ntet;
    n2t_ptr.assign(nn + 1, 0);
    for (int64_t k = 0; k < 4 * nt; ++k) n2t_ptr[p.tet[k] + 1]++;
    for (int64_t i = 0; i < nn; ++i) n2t_ptr[i + 1] += n2t_ptr[i];
    n2t.resize(4 * nt);
    {
        std::vector<int32_t> fill(n2t_ptr.begin(), n2t_ptr.end() - 1);
        for (int64_t t = 0; t < nt; ++t)
            for (int a = 0; a < 4; ++a) n2t[fill[p.tet[4 * t + a]]++] = int32_t(t * 4 + a);
    }
    // local surface ids of FEM nodes
    std::vector<int32_t> loc[2];
    for (int w = 0; w < 2; ++w) {
        loc[w].assign(nn, -1);
        for (int64_t i = 0; i < p.topo[w].nv; ++i) loc[w][p.topo[w].g[i]] = int32_t(i);
    }
    const int64_t off[2] = {nn, nn + p.topo[0].nv};
    // row patterns: the nodes of the tets at the row node, then the
    // coupling columns of the triangles at it (surface nodes), ascending
    std::vector<int32_t> rowptr(nn + 1, 0), rc;
    std::vector<int32_t> cols;
    for (int64_t a = 0; a < nn; ++a) {
        cols.clear();
        for (int32_t e = n2t_ptr[a]; e < n2t_ptr[a + 1]; ++e) {
            int32_t t = n2t[e] / 4;
            for (int b = 0; b < 4; ++b) cols.push_back(p.tet[4 * t + b]);
        }
        for (int w = 0; w < 2; ++w) {
            int32_t i = loc[w][a];
            if (i < 0) continue;
            const SurfaceTopo &S = p.topo[w];
            for (int32_t e = S.v2t_ptr[i]; e < S.v2t_ptr[i + 1]; ++e) {
                int32_t t = S.v2t[e] / 3;
                for (int b = 0; b < 3; ++b) cols.push_back(int32_t(off[w] + S.tri[3 * t + b]));
            }
        }
        std::sort(cols.begin(), cols.end());
        cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
        rc.insert(rc.end(), cols.begin(), cols.end());
        rowptr[a + 1] = int32_t(rc.size());
    }
    p.nnz_row = int64_t(rc.size());
    // sliced ELL: slice width = longest row of the slice; entry k of row
    // 64 q + l at sptr[q] + 64 k + l; padding: column = row, value 0
    const int64_t nsl = (nn + SLICE - 1) / SLICE;
    sptr.assign(nsl + 1, 0);
    for (int64_t q = 0; q < nsl; ++q) {
        int32_t w = 0;
        for (int64_t a = q * SLICE; a < std::min(nn, (q + 1) * SLICE); ++a) w = std::max(w, rowptr[a + 1] - rowptr[a]);
        PB_CHECK(int64_t(sptr[q]) + int64_t(SLICE) * w < (int64_t(1) << 31), PBFB_EINVAL,
                 "FEM block too large for 32-bit slice offsets");
        sptr[q + 1] = sptr[q] + SLICE * w;
    }
    col.assign(sptr[nsl], 0);
    std::vector<int32_t> pos(rc.size()); // row-pattern index -> stored slot
    for (int64_t q = 0; q < nsl; ++q) {
        const int32_t w = (sptr[q + 1] - sptr[q]) / SLICE;
        for (int l = 0; l < SLICE; ++l) {
            const int64_t a = q * SLICE + l;
            const int32_t len = a < nn ? rowptr[a + 1] - rowptr[a] : 0;
            for (int32_t k = 0; k < w; ++k) {
                const int64_t at = sptr[q] + int64_t(SLICE) * k + l;
                if (k < len) {
                    col[at] = rc[rowptr[a] + k];
                    pos[rowptr[a] + k] = int32_t(at);
                } else {
                    col[at] = a < nn ? int32_t(a) : 0;
                }
            }
        }
    }
    auto find = [&](int64_t row, int64_t c) {
        auto b = rc.begin() + rowptr[row], e = rc.begin() + rowptr[row + 1];
        auto it = std::lower_bound(b, e, int32_t(c));
        return pos[it - rc.begin()];
    };
    slot4.resize(4 * n2t.size());
    for (int64_t a = 0; a < nn; ++a)
        for (int32_t e = n2t_ptr[a]; e < n2t_ptr[a + 1]; ++e) {
            int32_t t = n2t[e] / 4;
            for (int b = 0; b < 4; ++b) slot4[4 * int64_t(e) + b] = find(a, p.tet[4 * t + b]);
        }
    diag.resize(nn);
    for (int64_t a = 0; a < nn; ++a) diag[a] = find(a, a);
    for (int w = 0; w < 2; ++w) {
        const SurfaceTopo &S = p.topo[w];
        cslot[w].resize(3 * S.v2t.size());
        for (int64_t i = 0; i < S.nv; ++i)
            for (int32_t e = S.v2t_ptr[i]; e < S.v2t_ptr[i + 1]; ++e) {
                int32_t t = S.v2t[e] / 3;
                for (int b = 0; b < 3; ++b) cslot[w][3 * int64_t(e) + b] = find(S.g[i], off[w] + S.tri[3 * t + b]);
            }
    }
}

// 3-ring of each vertex (vertices within three edges of a triangle path,
// itself included), ascending: the pattern of the near-field single layer
// from which the matrix-free preconditioner is built
void near_pattern(SurfaceTopo &S)
{
    if (!S.nf_ptr.empty()) return;
    std::vector<int32_t> mark(S.nv, -1), cur, next;
    S.nf_ptr.assign(S.nv + 1, 0);
    S.nf_col.clear();
    for (int64_t i = 0; i < S.nv; ++i) {
        cur.assign(1, int32_t(i));
        mark[i] = int32_t(i);
        for (int depth = 0; depth < 3; ++depth) {
            next = cur;
            for (int32_t j : cur)
                for (int32_t e = S.ring_ptr[j]; e < S.ring_ptr[j + 1]; ++e) {
                    const int32_t k = S.ring[e];
                    if (mark[k] != int32_t(i)) {
                        mark[k] = int32_t(i);
                        next.push_back(k);
                    }
                }
            cur.swap(next);
        }
        std::sort(cur.begin(), cur.end());
        S.nf_col.insert(S.nf_col.end(), cur.begin(), cur.end());
        S.nf_ptr[i + 1] = int32_t(S.nf_col.size());
    }
}

// In the Morton vertex order (operator indices): for each k the indices
// l > k within two rings of vertex mvert[k], ascending: every pair whose
// entry can receive a touching-pair block (a vertex on a triangle that shares
// a vertex with a triangle at the other)
void delta_pattern(SurfaceTopo &S)
{
    if (!S.d2_ptr.empty()) return;
    std::vector<int32_t> mark(S.nv, -1), cur;
    S.d2_ptr.assign(S.nv + 1, 0);
    S.d2_col.clear();
    for (int64_t k = 0; k < S.nv; ++k) {
        cur.clear();
        const int32_t i = S.mvert[k];
        for (int32_t e = S.ring_ptr[i]; e < S.ring_ptr[i + 1]; ++e) {
            const int32_t a = S.ring[e];
            for (int32_t f = S.ring_ptr[a]; f < S.ring_ptr[a + 1]; ++f) {
                const int32_t l = S.minv[S.ring[f]];
                if (l > k && mark[l] != int32_t(k)) {
                    mark[l] = int32_t(k);
                    cur.push_back(l);
                }
            }
        }
        std::sort(cur.begin(), cur.end());
        S.d2_col.insert(S.d2_col.end(), cur.begin(), cur.end());
        S.d2_ptr[k + 1] = int32_t(S.d2_col.size());
    }
}

} // namespace pbfb
