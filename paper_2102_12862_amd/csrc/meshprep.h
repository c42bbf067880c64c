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
};

bool prepare_mesh(const double *xyz, int64_t nv, const int32_t *tri, int64_t nc, const int32_t *seg,
                  const int32_t *tag, int64_t ns, bool renumber, HostMesh &M, std::string &err);

}  // namespace swe
