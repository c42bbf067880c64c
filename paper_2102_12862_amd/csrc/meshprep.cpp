// Host mesh preparation: validation, counter-clockwise fix, edge matching,
// boundary tags, FP64 geometry, Hilbert renumbering of cells.
//
// Follows the discretisation of the paper (section "Domain discretization"):
// a conforming triangulation, each cell with up to three neighbours across
// edges of length l and unit normal n pointing toward the neighbour.
#include "meshprep.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <unordered_map>
#include <utility>

namespace swe {

namespace {

// Hilbert index of (x, y) on a 2^16 x 2^16 grid.
uint32_t hilbert16(uint32_t x, uint32_t y) {
    uint32_t d = 0;
    const uint32_t n = 1u << 16;
    for (uint32_t s = n >> 1; s > 0; s >>= 1) {
        const uint32_t rx = (x & s) ? 1u : 0u;
        const uint32_t ry = (y & s) ? 1u : 0u;
        d += s * s * ((3u * rx) ^ ry);
        if (ry == 0) {
            if (rx == 1) {
                x = n - 1 - x;
                y = n - 1 - y;
            }
            std::swap(x, y);
        }
    }
    return d;
}

struct HalfEdge {
    int32_t hi;    // larger node id of the edge
    int32_t cell;  // original cell id
    int32_t k;     // local edge index
};

}  // namespace

bool prepare_mesh(const double *xyz, int64_t nv, const int32_t *tri, int64_t nc, const int32_t *seg,
                  const int32_t *tag, int64_t ns, bool renumber, HostMesh &M, std::string &err) {
    if (nv < 3 || nc < 1) { err = "empty mesh"; return false; }
    if (nc >= (int64_t)NBR_LIMIT || nv >= (int64_t)INT32_MAX) { err = "mesh too large (cells must be < 2^30)"; return false; }
    for (int64_t v = 0; v < nv; v++)
        if (!std::isfinite(xyz[3 * v]) || !std::isfinite(xyz[3 * v + 1]) || !std::isfinite(xyz[3 * v + 2])) {
            err = "non-finite node coordinate";
            return false;
        }
    M.nv = nv;
    M.nc = nc;
    std::vector<int32_t> t3((size_t)(3 * nc));
    std::vector<double> area0((size_t)nc), zb0((size_t)nc), cx((size_t)nc), cy((size_t)nc);
    for (int64_t i = 0; i < nc; i++) {
        int32_t a = tri[3 * i], b = tri[3 * i + 1], c = tri[3 * i + 2];
        if (a < 0 || b < 0 || c < 0 || a >= nv || b >= nv || c >= nv || a == b || b == c || a == c) {
            err = "bad triangle vertex index";
            return false;
        }
        const double *A = xyz + 3 * a, *B = xyz + 3 * b, *C = xyz + 3 * c;
        double cr = (B[0] - A[0]) * (C[1] - A[1]) - (B[1] - A[1]) * (C[0] - A[0]);
        if (cr < 0) {
            std::swap(b, c);
            cr = -cr;
        }
        if (!(cr > 0)) { err = "degenerate triangle"; return false; }
        t3[3 * i] = a; t3[3 * i + 1] = b; t3[3 * i + 2] = c;
        area0[i] = 0.5 * cr;
        zb0[i] = (xyz[3 * a + 2] + xyz[3 * b + 2] + xyz[3 * c + 2]) / 3.0;
        cx[i] = (xyz[3 * a] + xyz[3 * b] + xyz[3 * c]) / 3.0;
        cy[i] = (xyz[3 * a + 1] + xyz[3 * b + 1] + xyz[3 * c + 1]) / 3.0;
    }
    // half-edges bucketed by their smaller node (counting sort, O(N))
    std::vector<int64_t> off((size_t)nv + 1, 0);
    for (int64_t i = 0; i < nc; i++)
        for (int k = 0; k < 3; k++) {
            const int32_t p = t3[3 * i + k], q = t3[3 * i + (k + 1) % 3];
            off[(size_t)std::min(p, q) + 1]++;
        }
    for (int64_t v = 0; v < nv; v++) off[v + 1] += off[v];
    std::vector<HalfEdge> he((size_t)(3 * nc));
    {
        std::vector<int64_t> fill(off.begin(), off.end() - 1);
        for (int64_t i = 0; i < nc; i++)
            for (int k = 0; k < 3; k++) {
                const int32_t p = t3[3 * i + k], q = t3[3 * i + (k + 1) % 3];
                he[(size_t)fill[std::min(p, q)]++] = HalfEdge{std::max(p, q), (int32_t)i, k};
            }
    }
    // per segment its tag and its first node (the direction a segment on
    // interior edges gives: the cell on its left is the upstream side of an
    // internal rating curve)
    std::unordered_map<uint64_t, std::pair<int32_t, int32_t>> segtag;
    segtag.reserve((size_t)ns * 2 + 1);
    for (int64_t s = 0; s < ns; s++) {
        const int32_t p = seg[2 * s], q = seg[2 * s + 1];
        if (p < 0 || q < 0 || p >= nv || q >= nv || p == q) { err = "bad boundary segment"; return false; }
        const uint64_t key = ((uint64_t)std::min(p, q) << 32) | (uint32_t)std::max(p, q);
        if (!segtag.emplace(key, std::make_pair(tag[s], p)).second) { err = "duplicate boundary segment"; return false; }
    }
    // neighbour of every (old cell, local edge): old neighbour id, or -1 - boundary id
    std::vector<int32_t> link((size_t)(3 * nc));
    std::vector<int32_t> itag0((size_t)(3 * nc), -1);  // tag of a tagged interior edge
    std::vector<uint8_t> up0((size_t)(3 * nc), 0);     // the cell is on the left of that edge's segment
    std::vector<int32_t> btag;
    int64_t matched = 0, ne = 0;
    for (int64_t v = 0; v < nv; v++) {
        HalfEdge *b = he.data() + off[v], *e = he.data() + off[v + 1];
        std::sort(b, e, [](const HalfEdge &x, const HalfEdge &y) {
            return x.hi != y.hi ? x.hi < y.hi : x.cell < y.cell;
        });
        for (HalfEdge *g = b; g < e;) {
            HalfEdge *h = g + 1;
            while (h < e && h->hi == g->hi) h++;
            const int64_t cnt = h - g;
            if (cnt > 2) { err = "non-conforming edge shared by 3+ triangles"; return false; }
            ne++;
            if (cnt == 2) {
                const int32_t c1 = g[0].cell, k1 = g[0].k, c2 = g[1].cell, k2 = g[1].k;
                // the two cells must traverse the edge in opposite directions
                const int32_t q1 = t3[3 * c1 + (k1 + 1) % 3];
                if (t3[3 * c2 + k2] != q1) { err = "inconsistent orientation (overlapping triangles)"; return false; }
                link[3 * c1 + k1] = c2;
                link[3 * c2 + k2] = c1;
                const uint64_t key = ((uint64_t)v << 32) | (uint32_t)g->hi;
                auto it = segtag.find(key);
                if (it != segtag.end()) {
                    itag0[3 * c1 + k1] = itag0[3 * c2 + k2] = it->second.first;
                    // a counter-clockwise cell walking the edge in the
                    // segment's direction lies on the segment's left
                    up0[3 * c1 + k1] = t3[3 * c1 + k1] == it->second.second;
                    up0[3 * c2 + k2] = t3[3 * c2 + k2] == it->second.second;
                    matched++;
                }
            } else {
                const uint64_t key = ((uint64_t)v << 32) | (uint32_t)g->hi;
                auto it = segtag.find(key);
                int32_t tg = -1;
                if (it != segtag.end()) {
                    tg = it->second.first;
                    matched++;
                }
                link[3 * g->cell + g->k] = -1 - (int32_t)btag.size();
                btag.push_back(tg);
            }
            g = h;
        }
    }
    if (matched != ns) { err = "segment is not an edge of the mesh"; return false; }
    M.iw_tags.clear();
    for (int32_t tg : itag0)
        if (tg >= 0 && std::find(M.iw_tags.begin(), M.iw_tags.end(), tg) == M.iw_tags.end()) {
            if ((int)M.iw_tags.size() == MAX_IW_TAGS) { err = "at most 31 tags on interior edges"; return false; }
            M.iw_tags.push_back(tg);
        }
    M.ne = ne;
    M.nb = (int64_t)btag.size();

    // renumbering: Hilbert order of centroids on a square box (isotropic)
    M.perm.resize((size_t)nc);
    for (int64_t i = 0; i < nc; i++) M.perm[i] = (int32_t)i;
    if (renumber && nc > 1) {
        double x0 = cx[0], x1 = cx[0], y0 = cy[0], y1 = cy[0];
        for (int64_t i = 1; i < nc; i++) {
            x0 = std::min(x0, cx[i]); x1 = std::max(x1, cx[i]);
            y0 = std::min(y0, cy[i]); y1 = std::max(y1, cy[i]);
        }
        const double ext = std::max(x1 - x0, y1 - y0);
        const double sc = ext > 0 ? 65535.0 / ext : 0.0;
        std::vector<uint64_t> key((size_t)nc);
        for (int64_t i = 0; i < nc; i++) {
            const uint32_t hx = (uint32_t)std::min(65535.0, std::max(0.0, (cx[i] - x0) * sc));
            const uint32_t hy = (uint32_t)std::min(65535.0, std::max(0.0, (cy[i] - y0) * sc));
            key[i] = ((uint64_t)hilbert16(hx, hy) << 32) | (uint32_t)i;
        }
        std::sort(key.begin(), key.end());
        for (int64_t p = 0; p < nc; p++) M.perm[p] = (int32_t)(key[p] & 0xffffffffu);
    }
    M.inv.resize((size_t)nc);
    for (int64_t p = 0; p < nc; p++) M.inv[M.perm[p]] = (int32_t)p;

    // device-order arrays
    M.area.resize((size_t)nc);
    M.zb.resize((size_t)nc);
    M.lx.resize((size_t)(3 * nc));
    M.ly.resize((size_t)(3 * nc));
    M.nbr.resize((size_t)(3 * nc));
    M.iw_slot.assign((size_t)(3 * nc), -1);
    M.iw_up.assign((size_t)(3 * nc), 0);
    M.slot_tag.clear();
    M.slot_len.clear();
    M.slot_cell.clear();
    for (int64_t p = 0; p < nc; p++) {
        const int32_t i = M.perm[p];
        M.area[p] = area0[i];
        M.zb[p] = zb0[i];
        for (int k = 0; k < 3; k++) {
            const int32_t a = t3[3 * i + k], b = t3[3 * i + (k + 1) % 3];
            const double dx = xyz[3 * b] - xyz[3 * a], dy = xyz[3 * b + 1] - xyz[3 * a + 1];
            // l * n for a counter-clockwise cell: (dy, -dx); the neighbour walks
            // the edge the other way and stores the exact negation
            M.lx[3 * p + k] = dy;
            M.ly[3 * p + k] = -dx;
            const int32_t L = link[3 * i + k];
            if (itag0[3 * i + k] >= 0) {
                M.iw_slot[3 * p + k] = (int32_t)(std::find(M.iw_tags.begin(), M.iw_tags.end(), itag0[3 * i + k]) -
                                                 M.iw_tags.begin());
                M.iw_up[3 * p + k] = up0[3 * i + k];
            }
            if (L >= 0) {
                int32_t code = M.inv[L];
                if (i > L) code |= NBR_FLIP_BIT;  // canonical left cell = smaller original id
                M.nbr[3 * p + k] = code;
            } else {
                const int32_t slot = (int32_t)M.slot_tag.size();
                M.slot_tag.push_back(btag[-1 - L]);
                M.slot_len.push_back(std::sqrt(dx * dx + dy * dy));
                M.slot_cell.push_back((int32_t)p);
                M.nbr[3 * p + k] = -1 - slot;
            }
        }
    }
    return true;
}

bool build_tile_edges(const HostMesh &M, int tile, std::vector<TileEdge> &edges, std::vector<int32_t> &eoff) {
    if (tile < 64 || tile > MAX_TILE) return false;
    const int64_t n = M.nc;
    const int64_t ntiles = (n + tile - 1) / tile;
    edges.clear();
    edges.reserve((size_t)(n * 7 / 4 + ntiles * 64));
    eoff.assign((size_t)ntiles + 1, 0);
    std::vector<TileEdge> remote, boundary;
    for (int64_t t = 0; t < ntiles; t++) {
        eoff[t] = (int32_t)edges.size();
        remote.clear();
        boundary.clear();
        const int64_t p0 = t * tile, p1 = std::min(n, p0 + tile);
        for (int64_t p = p0; p < p1; p++) {
            for (int k = 0; k < 3; k++) {
                const int32_t code = M.nbr[3 * p + k];
                TileEdge e;
                e.lx = M.lx[3 * p + k];
                e.ly = M.ly[3 * p + k];
                int32_t w0 = (int32_t)(p - p0) | (k << 10);
                const int32_t iw = M.iw_slot[3 * p + k];
                if (code >= 0) {
                    const int32_t q = code & (NBR_FLIP_BIT - 1);
                    if (code & NBR_FLIP_BIT) w0 |= 1 << 16;
                    if (iw >= 0) {
                        // a tagged interior edge: one record per side, bit 17
                        // set on the side left of the tag's segment
                        w0 |= (EDGE_REMOTE << 14) | (int32_t)((uint32_t)(iw + 1) << 27) |
                              ((int32_t)M.iw_up[3 * p + k] << 17);
                        e.w1 = q;
                    } else if (q >= p0 && q < p1) {
                        if (q < p) continue;  // emitted from the other cell
                        int kb = -1;
                        for (int k2 = 0; k2 < 3; k2++) {
                            const int32_t c2 = M.nbr[3 * q + k2];
                            if (c2 >= 0 && (c2 & (NBR_FLIP_BIT - 1)) == p) kb = k2;
                        }
                        if (kb < 0) return false;
                        w0 |= (kb << 12) | (EDGE_LOCAL << 14) | (int32_t)((q - p0) << 17);
                        e.w1 = q;
                    } else {
                        w0 |= EDGE_REMOTE << 14;
                        e.w1 = q;
                    }
                } else {
                    w0 |= EDGE_BOUNDARY << 14;
                    e.w1 = -1 - code;
                }
                e.w0 = w0;
                const int kind = (w0 >> 14) & 3;
                if (kind == EDGE_LOCAL)
                    edges.push_back(e);
                else if (kind == EDGE_REMOTE)
                    remote.push_back(e);
                else
                    boundary.push_back(e);
            }
        }
        // local edges first, then remote ones by neighbour (gathers in
        // address order), then boundary edges: a wave then mostly runs one
        // kind of edge
        std::stable_sort(remote.begin(), remote.end(),
                         [](const TileEdge &x, const TileEdge &y) { return x.w1 < y.w1; });
        edges.insert(edges.end(), remote.begin(), remote.end());
        edges.insert(edges.end(), boundary.begin(), boundary.end());
    }
    eoff[ntiles] = (int32_t)edges.size();
    return edges.size() < (size_t)INT32_MAX;
}

std::string check_tile_edges(const HostMesh &M, int tile, const std::vector<TileEdge> &edges,
                             const std::vector<int32_t> &eoff) {
    const int64_t n = M.nc;
    const int64_t ntiles = (n + tile - 1) / tile;
    if ((int64_t)eoff.size() != ntiles + 1 || eoff[0] != 0 || eoff[ntiles] != (int32_t)edges.size())
        return "bad tile offsets";
    std::vector<int8_t> seen((size_t)(3 * n), 0);
    for (int64_t t = 0; t < ntiles; t++) {
        if (eoff[t] > eoff[t + 1]) return "decreasing tile offsets";
        const int64_t p0 = t * tile;
        for (int32_t e = eoff[t]; e < eoff[t + 1]; e++) {
            const TileEdge &E = edges[e];
            const int a = E.w0 & 1023, ka = (E.w0 >> 10) & 3, kb = (E.w0 >> 12) & 3, kind = (E.w0 >> 14) & 3;
            const int flip = (E.w0 >> 16) & 1;
            const int64_t pa = p0 + a;
            if (a >= tile || pa >= n || ka > 2) return "edge cell outside its tile";
            if (E.lx != M.lx[3 * pa + ka] || E.ly != M.ly[3 * pa + ka]) return "edge geometry differs from its cell";
            const int32_t code = M.nbr[3 * pa + ka];
            const int iwf = (int)(((uint32_t)E.w0 >> 27) & 31);
            if (iwf != M.iw_slot[3 * pa + ka] + 1) return "interior-tag index mismatch";
            if (iwf && ((E.w0 >> 17) & 1) != M.iw_up[3 * pa + ka]) return "interior-tag side mismatch";
            if (iwf && ((E.w0 >> 18) & 511)) return "stray bits in a tagged interior record";
            seen[3 * pa + ka]++;
            if (kind == EDGE_BOUNDARY) {
                if (code >= 0 || E.w1 != -1 - code) return "boundary edge mismatch";
            } else {
                if (code < 0) return "interior edge on a boundary slot";
                const int32_t q = code & (NBR_FLIP_BIT - 1);
                if (flip != ((code & NBR_FLIP_BIT) ? 1 : 0)) return "orientation flag mismatch";
                if (E.w1 != q) return "neighbour id mismatch";
                const bool local = q >= p0 && q < std::min(n, p0 + tile) && !iwf;
                if ((kind == EDGE_LOCAL) != local) return "local/remote classification wrong";
                if (kind == EDGE_LOCAL) {
                    const int b = (E.w0 >> 17) & 1023;
                    if (p0 + b != q || kb > 2) return "local neighbour index mismatch";
                    if ((M.nbr[3 * q + kb] & (NBR_FLIP_BIT - 1)) != pa || M.nbr[3 * q + kb] < 0)
                        return "neighbour's local edge mismatch";
                    if (M.lx[3 * q + kb] != -E.lx || M.ly[3 * q + kb] != -E.ly) return "edge normals not opposite";
                    seen[3 * q + kb]++;
                }
            }
        }
    }
    for (int64_t k = 0; k < 3 * n; k++)
        if (seen[k] != 1) return "a cell edge is covered " + std::to_string((int)seen[k]) + " times";
    return "";
}

}  // namespace swe
