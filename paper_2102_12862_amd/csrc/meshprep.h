// Host mesh preparation (validation, edge matching, geometry, renumbering).
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

namespace swe {

constexpr int32_t NBR_LIMIT = 1 << 30;  // cells per mesh (neighbour ids carry a flag in bit 30)
constexpr int32_t NBR_FLIP_BIT = 1 << 30;

struct HostMesh {
    int64_t nv = 0, nc = 0, ne = 0, nb = 0;
    std::vector<int32_t> perm;   // device order -> input order
    std::vector<int32_t> inv;    // input order -> device order
    std::vector<double> area;    // device order
    std::vector<double> zb;      // cell bed = mean of node elevations
    std::vector<double> lx, ly;  // 3 per cell: l * outward unit normal
    std::vector<int32_t> nbr;    // 3 per cell: device id | flip bit, or -1 - slot
    std::vector<int32_t> slot_tag;   // per boundary slot (slot order = device cell, local edge)
    std::vector<double> slot_len;
    std::vector<int32_t> slot_cell;
    // tagged interior edges (internal conditions): per (device cell, local
    // edge) the index of its tag in iw_tags, or -1; at most 31 distinct tags
    std::vector<int32_t> iw_slot;
    std::vector<int32_t> iw_tags;
    // per (device cell, local edge) of a tagged interior edge: 1 when the
    // cell lies on the left of the edge's segment (its first node to its
    // second), the upstream side of an internal rating curve
    std::vector<uint8_t> iw_up;
};
constexpr int MAX_IW_TAGS = 31;

// One edge of a tile (a block of `tile` consecutive cells), stored once per
// tile: an edge between two cells of the tile appears once, an edge to a
// cell of another tile or to the boundary appears in the tile of its cell.
// Within a tile the list holds the local edges first, then the remote ones
// in order of the other cell, then the boundary edges.
//   w0: bits 0-9 local cell a, 10-11 its local edge ka, 12-13 the other
//       cell's local edge kb, 14-15 kind (0 both cells in the tile, 1 other
//       cell in another tile, 2 boundary), bit 16 set when a is the right
//       cell of the edge's canonical orientation, bits 17-26 local cell b,
//       bits 27-31 one plus the interior-tag index of a tagged interior edge
//       (such an edge is stored once per side, as kind 1, even when both
//       cells are in the tile, so that each side can become a wall; its bit
//       17 is set on the side left of the tag's segment)
//   w1: kind 1: device id of the other cell; kind 2: boundary slot
//   lx, ly: l * n with n the outward normal of a
enum : int32_t { EDGE_LOCAL = 0, EDGE_REMOTE = 1, EDGE_BOUNDARY = 2 };
struct TileEdge {
    int32_t w0, w1;
    double lx, ly;
};
constexpr int MAX_TILE = 1024;

bool build_tile_edges(const HostMesh &M, int tile, std::vector<TileEdge> &edges, std::vector<int32_t> &eoff);
// Checks that the tile edge lists cover every (cell, local edge) exactly once
// with consistent indices, orientation and geometry; returns an empty string
// or the first problem found.
std::string check_tile_edges(const HostMesh &M, int tile, const std::vector<TileEdge> &edges,
                             const std::vector<int32_t> &eoff);

bool prepare_mesh(const double *xyz, int64_t nv, const int32_t *tri, int64_t nc, const int32_t *seg,
                  const int32_t *tag, int64_t ns, bool renumber, HostMesh &M, std::string &err);

}  // namespace swe
