// Host construction of the compact row layout and of the per-cell link words
// (what the kernels of step.hpp and step27.hpp address through), kept free of
// device calls so that it can be built and checked on its own.
#pragma once
#include <cstdint>
#include <vector>

#include "lbm.h"
#include "step.hpp"
#include "step27.hpp"

namespace lbmrt {

using namespace lbm;

// Cells per population plane: the compact count rounded up to a multiple of 64,
// so that every plane starts on a 128-byte boundary (16-bit storage; 256 bytes
// for FP32) and a wave's access to one plane covers whole cache lines.  The
// padding slots are never read or written.
inline int64_t plane_cells(int64_t nc) { return (nc + 63) & ~int64_t(63); }
// Wave records (lbm::WaveInfo) of the D3Q19 step: one per 64 compact cells of
// the largest step grid (blocks of 256).
inline int64_t wave_records(int64_t nc) { return (nc + 255) / 256 * 4; }

// Rows of the compact layout: every (y, z) line holding fluid, ordered by z
// then y, with the x range from its first to its last fluid cell.
struct Rows {
  std::vector<int> y, z, x0, x1;
  std::vector<int64_t> cb;  // compact start of each row
  int64_t nc = 0;           // compact cells (fluid + dead)
  int64_t nf = 0;           // fluid cells
};

// The host side of a context's layout: the box, the rows, the per-cell and
// per-row tables uploaded to the workspace, and the fluid-cell lists.
struct HostLayout {
  int nx = 0, ny = 0, nz = 0;
  int periodic[3] = {0, 0, 0};
  int outlet = 0;                 // outflow kind on x = nx - 1 (lbm_open.outlet)
  int xbits = 1;                  // position code = (row << xbits) | x
  int64_t nf = 0;                 // fluid cells
  int64_t nc = 0;                 // compact cells (fluid + dead)
  int64_t nrow = 0;
  int64_t nreg = 0;               // region cells
  Rows rows;
  std::vector<uint8_t> solid;     // the mask, box layout
  std::vector<uint32_t> code;     // per compact cell
  std::vector<uint32_t> rowbox;   // box index of (x = 0) of each row
  std::vector<int> delta;         // [nrow][8]: compact start - first x of the neighbour row of pair k
  std::vector<int> rel;           // [nrow][8]: delta minus (compact start - first x) of the row itself
  std::vector<int64_t> fluid_box; // box index per fluid cell (ascending)
  std::vector<int64_t> fluid_c;   // compact index per fluid cell
  std::vector<uint8_t> region_f;  // per fluid cell
  std::vector<uint8_t> openface;  // per fluid cell: 1 inflow, 2 outflow
};

inline Rows find_rows(const lbm_grid& g, const uint8_t* solid) {
  Rows r;
  const int nx = g.nx;
  for (int z = 0; z < g.nz; ++z)
    for (int y = 0; y < g.ny; ++y) {
      const uint8_t* line = solid + ((size_t)z * g.ny + y) * nx;
      int lo = -1, hi = -1;
      for (int x = 0; x < nx; ++x)
        if (!line[x]) {
          if (lo < 0) lo = x;
          hi = x;
          r.nf += 1;
        }
      if (lo < 0) continue;
      r.y.push_back(y); r.z.push_back(z); r.x0.push_back(lo); r.x1.push_back(hi + 1);
      r.cb.push_back(r.nc);
      r.nc += hi + 1 - lo;
    }
  return r;
}

inline int xbits_for(int nx) {
  int b = 1;
  while ((1 << b) < nx) ++b;
  return b;
}


// Fill the layout of a box with the given mask (nonzero = solid), optional
// region mask, and open faces (inflow on x = 0, outflow kind on x = nx - 1).
inline void build_host_layout(HostLayout& L, const lbm_grid& g, const uint8_t* solid, const uint8_t* region,
                              bool inlet, int outlet) {
  L.nx = g.nx; L.ny = g.ny; L.nz = g.nz;
  for (int a = 0; a < 3; ++a) L.periodic[a] = g.periodic[a] != 0;
  L.outlet = outlet;
  const size_t nbox = (size_t)g.nx * g.ny * g.nz;
  L.solid.assign(solid, solid + nbox);
  L.rows = find_rows(g, solid);
  L.nf = L.rows.nf;
  L.nc = L.rows.nc;
  L.nrow = (int64_t)L.rows.y.size();
  const int nx = g.nx, xb = xbits_for(nx);
  L.xbits = xb;
  L.code.assign(L.nc, 0u);
  L.rowbox.assign(L.nrow, 0u);
  L.delta.assign((size_t)L.nrow * 8, 0);
  L.rel.assign((size_t)L.nrow * 8, 0);
  std::vector<int64_t> rowid((size_t)g.ny * g.nz, -1);
  L.fluid_box.clear(); L.fluid_c.clear(); L.region_f.clear(); L.openface.clear();
  L.fluid_box.reserve(L.nf);
  L.fluid_c.reserve(L.nf);
  L.nreg = 0;
  for (int64_t r = 0; r < L.nrow; ++r) {
    const int y = L.rows.y[r], z = L.rows.z[r];
    rowid[(size_t)z * g.ny + y] = r;
    const size_t base = ((size_t)z * g.ny + y) * nx;
    L.rowbox[r] = (uint32_t)base;
    for (int x = L.rows.x0[r]; x < L.rows.x1[r]; ++x) {
      const int64_t ci = L.rows.cb[r] + x - L.rows.x0[r];
      L.code[ci] = ((uint32_t)r << xb) | (uint32_t)x;
      const size_t b = base + x;
      if (solid[b]) continue;
      L.fluid_box.push_back((int64_t)b);
      L.fluid_c.push_back(ci);
      L.region_f.push_back(region && region[b] ? 1 : 0);
      uint8_t of = 0;
      if (inlet && x == 0) of = 1;
      else if (outlet && x == nx - 1) of = 2;
      L.openface.push_back(of);
      L.nreg += (region && region[b]) ? 1 : 0;
    }
  }
  // neighbour-row deltas: the row (y - cy, z - cz) of pair k, wrapped on periodic axes
  for (int64_t r = 0; r < L.nrow; ++r) {
    for (int k = 1; k < NPAIR; ++k) {
      int sy = L.rows.y[r] - PCY[k], sz = L.rows.z[r] - PCZ[k];
      if (g.periodic[1]) sy = (sy + g.ny) % g.ny;
      if (g.periodic[2]) sz = (sz + g.nz) % g.nz;
      if (sy < 0 || sy >= g.ny || sz < 0 || sz >= g.nz) continue;
      const int64_t rr = rowid[(size_t)sz * g.ny + sy];
      if (rr < 0) continue;
      L.delta[(size_t)r * 8 + (k - 1)] = (int)(L.rows.cb[rr] - L.rows.x0[rr]);
      // (x, row rr) sits at c + rel from (x, row r) = c
      L.rel[(size_t)r * 8 + (k - 1)] =
          (int)((L.rows.cb[rr] - L.rows.x0[rr]) - (L.rows.cb[r] - L.rows.x0[r]));
    }
  }
}

// Link word of every compact cell (see step.hpp): dead flag, bounce-back mask
// of the pulls, uniform-neighbour-porosity flag, open-face role, region,
// open-face unknowns.  Returns the number of region cells on the wall (a wall
// link that is not an open-face unknown, and a nonzero weighted link sum).
inline int64_t build_links(const HostLayout& c, const std::vector<float>& phib, std::vector<uint32_t>& links) {
  int64_t nwss = 0;
  const int nx = c.nx, ny = c.ny, nz = c.nz;
  const int per[3] = {c.periodic[0] != 0, c.periodic[1] != 0, c.periodic[2] != 0};
  const int dims[3] = {nx, ny, nz};
  links.assign(c.nc, LK_DEAD);
  for (int64_t k = 0; k < c.nf; ++k) {
    const int64_t b = c.fluid_box[k];
    const int X[3] = {(int)(b % nx), (int)((b / nx) % ny), (int)(b / ((int64_t)nx * ny))};
    uint32_t lk = 0;
    bool uni = true;
    const float ph = phib[b];
    uint32_t unk = 0;
    int m[3] = {0, 0, 0};  // sum over wall links x + c_j of 36 w_j c_j
    for (int i = 1; i < Q; ++i) {
      const int cv[3] = {CX[i], CY[i], CZ[i]};
      for (int sgn = -1; sgn <= 1; sgn += 2) {  // -1: pull source x - c_i; +1: neighbour x + c_i
        int s[3];
        bool out = false, out_yz = false;
        for (int a = 0; a < 3; ++a) {
          s[a] = X[a] + sgn * cv[a];
          if (s[a] < 0 || s[a] >= dims[a]) {
            if (per[a]) s[a] = (s[a] + dims[a]) % dims[a];
            else { out = true; if (a > 0) out_yz = true; }
          }
        }
        const int64_t sb = out ? -1 : (int64_t)s[0] + (int64_t)nx * ((int64_t)s[1] + (int64_t)ny * s[2]);
        const bool wall = out || c.solid[sb];
        if (sgn < 0) {
          if (wall) lk |= 1u << i;
          // open-face unknown: the source lies beyond the inflow/outflow face only
          const bool open = out && !out_yz && c.openface[k];
          if (open) {
            const int* xs = c.openface[k] == 1 ? XIN : XOUT;
            for (int j = 0; j < 5; ++j)
              if (xs[j] == i) unk |= 1u << j;
          }
          if (wall && !open)
            for (int a = 0; a < 3; ++a) m[a] -= (int)kw(i) * cv[a];
        } else if (!wall && phib[sb] != ph) {
          uni = false;
        }
      }
    }
    if (uni) lk |= LK_UNI;
    // interior: every pull source is fluid and none wraps around x
    if ((lk & 0x7fffeu) == 0 && !(per[0] && (X[0] == 0 || X[0] == nx - 1))) lk |= LK_INR;
    if (c.openface[k] == 1) lk |= LK_IN;
    if (c.openface[k] == 2) lk |= LK_OUT;
    // -x neighbour of an extrapolation-outflow cell
    if (c.outlet == 2 && X[0] == nx - 2 && !c.solid[b + 1]) lk |= LK_UPS;
    if (c.region_f[k]) lk |= LK_REG;
    lk |= unk << LK_UNK;
    links[c.fluid_c[k]] = lk;
    if (c.region_f[k] && (m[0] | m[1] | m[2]) != 0) ++nwss;
  }
  return nwss;
}

// The 64-bit link words of the D3Q27 kernels (layout in step27.hpp); returns
// the number of region cells on the wall.
inline int64_t build_links27(const HostLayout& c, const std::vector<float>& phib, std::vector<uint64_t>& links) {
  namespace L = q27;
  const int nx = c.nx, ny = c.ny, nz = c.nz;
  const int per[3] = {c.periodic[0] != 0, c.periodic[1] != 0, c.periodic[2] != 0};
  const int dims[3] = {nx, ny, nz};
  int64_t nwss = 0;
  links.assign(c.nc, L::L_DEAD);
  for (int64_t k = 0; k < c.nf; ++k) {
    const int64_t b = c.fluid_box[k];
    const int X[3] = {(int)(b % nx), (int)((b / nx) % ny), (int)(b / ((int64_t)nx * ny))};
    uint64_t lk = 0;
    bool uni = true;
    const float ph = phib[b];
    uint64_t unk = 0;
    int m[3] = {0, 0, 0};
    for (int i = 1; i < L::Q; ++i) {
      const int cv[3] = {L::CX[i], L::CY[i], L::CZ[i]};
      for (int sgn = -1; sgn <= 1; sgn += 2) {  // -1: pull source x - c_i; +1: neighbour x + c_i
        int sidx[3];
        bool out = false, out_yz = false;
        for (int a = 0; a < 3; ++a) {
          sidx[a] = X[a] + sgn * cv[a];
          if (sidx[a] < 0 || sidx[a] >= dims[a]) {
            if (per[a]) sidx[a] = (sidx[a] + dims[a]) % dims[a];
            else { out = true; if (a > 0) out_yz = true; }
          }
        }
        const int64_t sb = out ? -1 : (int64_t)sidx[0] + (int64_t)nx * ((int64_t)sidx[1] + (int64_t)ny * sidx[2]);
        const bool wall = out || c.solid[sb];
        if (sgn < 0) {
          if (wall) lk |= 1ull << i;
          const bool open = out && !out_yz && c.openface[k];
          if (open) {
            const int* xs = c.openface[k] == 1 ? L::XIN : L::XOUT;
            for (int j = 0; j < L::NX; ++j)
              if (xs[j] == i) unk |= 1ull << j;
          }
          if (wall && !open)
            for (int a = 0; a < 3; ++a) m[a] -= L::kw(i) * cv[a];
        } else if (!wall && phib[sb] != ph) {
          uni = false;
        }
      }
    }
    if (uni) lk |= L::L_UNI;
    if (c.openface[k] == 1) lk |= L::L_IN;
    if (c.openface[k] == 2) lk |= L::L_OUT;
    if (c.outlet == 2 && X[0] == nx - 2 && !c.solid[b + 1]) lk |= L::L_UPS;
    if (c.region_f[k]) lk |= L::L_REG;
    lk |= unk << L::L_UNK;
    links[c.fluid_c[k]] = lk;
    if (c.region_f[k] && (m[0] | m[1] | m[2]) != 0) ++nwss;
  }
  return nwss;
}

}  // namespace lbmrt
