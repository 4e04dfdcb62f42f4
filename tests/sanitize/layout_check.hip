// Host-side check of the compact row layout and the link words that the step
// kernels address through, on seeded random boxes (extents 1..12, random
// periodic axes, open faces, solids, porosity and region).  Built with
// AddressSanitizer and UndefinedBehaviorSanitizer on the host; every table
// access of the check is bounds-checked.  For every fluid cell and direction
// of D3Q19 and D3Q27 it recomputes, by brute force over the box, where the pull
// source lies, and compares it with the layout:
//   - bounce-back bit of the link word <=> the source is solid or outside a
//     non-periodic face;
//   - otherwise the compact index the kernels form (x - c_x, wrapped on a
//     periodic x axis, plus the neighbour-row delta of the pair (c_y, c_z))
//     lies in [0, n_compact), is a fluid cell, and its position code decodes to
//     the source;
//   - byte offsets of every population slot stay below 2^32;
//   - uniform-neighbour-porosity, interior, open-face and unknown flags;
//   - interior cells: the source formed from the row offsets, c + rel[row][pair]
//     - c_x (the plain-wave path of the D3Q19 FP32 step), is the same compact
//     index (checked for both velocity sets);
//   - the row that the step derives for each lane of a 64-cell wave from the
//     wave's first row and its row-start bits is the cell's row.
// Exit status 0 when every check holds.
#include <cstdio>
#include <random>
#include <vector>

#include "layout.hpp"

using namespace lbmrt;

namespace {

int g_fail = 0;
long g_inr = 0;  // interior-path sources checked
void expect(bool ok, const char* what, int seed, long cell, int dir) {
  if (ok) return;
  if (g_fail < 20) std::printf("FAIL seed %d cell %ld dir %d: %s\n", seed, cell, dir, what);
  ++g_fail;
}

template <class LinkT, int NQ, class Dirs>
void check_links(const HostLayout& L, const std::vector<float>& phib, const std::vector<LinkT>& links,
                 const Dirs& cv, const int (&opp)[NQ], const int (&pk)[NQ], LinkT dead, LinkT uni_bit, LinkT in_bit,
                 LinkT out_bit, int unk_shift, const int* xin, const int* xout, int nx_face, LinkT inr_bit,
                 int seed) {
  const int dims[3] = {L.nx, L.ny, L.nz};
  const uint32_t xmask = (1u << L.xbits) - 1u;
  for (int64_t c = 0; c < L.nc; ++c) {
    const LinkT lk = links.at(c);
    const uint32_t code = L.code.at(c);
    const int64_t row = code >> L.xbits;
    const int x = (int)(code & xmask);
    expect(row >= 0 && row < L.nrow, "row of position code", seed, (long)c, -1);
    if (row < 0 || row >= L.nrow) continue;
    expect(x >= L.rows.x0.at(row) && x < L.rows.x1.at(row), "x inside the row's range", seed, (long)c, -1);
    expect(L.rows.cb.at(row) + x - L.rows.x0.at(row) == c, "compact index of the position code", seed, (long)c, -1);
    const int64_t b = (int64_t)L.rowbox.at(row) + x;
    const bool is_solid = L.solid.at(b) != 0;
    expect(((lk & dead) != 0) == is_solid, "dead flag <=> solid", seed, (long)c, -1);
    if (is_solid) continue;
    const int X[3] = {x, L.rows.y.at(row), L.rows.z.at(row)};
    const bool openf = x == 0 ? (lk & in_bit) != 0 : (x == L.nx - 1 ? (lk & out_bit) != 0 : false);
    bool uni = true, any_wall = false;
    int64_t rel_src[NQ], true_src[NQ];  // per direction: source from the row offsets, and the true one
    for (int i = 0; i < NQ; ++i) rel_src[i] = true_src[i] = -1;
    for (int i = 1; i < NQ; ++i) {
      // the pull source x - c_i, by brute force
      int s[3];
      bool out = false, out_yz = false;
      for (int a = 0; a < 3; ++a) {
        s[a] = X[a] - cv[i][a];
        if (s[a] < 0 || s[a] >= dims[a]) {
          if (L.periodic[a]) s[a] = (s[a] + dims[a]) % dims[a];
          else { out = true; out_yz = out_yz || a > 0; }
        }
      }
      const int64_t sb = out ? -1 : (int64_t)s[0] + (int64_t)L.nx * ((int64_t)s[1] + (int64_t)L.ny * s[2]);
      const bool wall = out || L.solid.at(sb) != 0;
      any_wall = any_wall || wall;
      expect(((lk >> i) & 1u) == (wall ? 1u : 0u), "bounce-back bit <=> source solid or outside", seed, (long)c, i);
      // the open-face unknowns
      if (out && !out_yz && openf) {
        const int* xs = x == 0 ? xin : xout;
        int j = -1;
        for (int k = 0; k < nx_face; ++k) if (xs[k] == i) j = k;
        expect(j >= 0 && ((lk >> (unk_shift + j)) & 1u), "open-face unknown bit", seed, (long)c, i);
      }
      if (!wall) {
        // the kernels' compact index of the source
        int xs = x - cv[i][0];
        if (L.periodic[0]) xs = (xs + L.nx) % L.nx;
        const int k = pk[i];
        const int64_t dl = k == 0 ? (int64_t)c - x : (int64_t)L.delta.at((size_t)row * 8 + (k - 1));
        const int64_t src = xs + dl;
        expect(src >= 0 && src < L.nc, "source compact index in range", seed, (long)c, i);
        if (src >= 0 && src < L.nc) {
          const uint32_t sc = L.code.at(src);
          const int64_t srow = sc >> L.xbits;
          expect(srow < L.nrow && (int)(sc & xmask) == s[0] && L.rows.y.at(srow) == s[1] && L.rows.z.at(srow) == s[2],
                 "source position code", seed, (long)c, i);
          expect(!(links.at(src) & dead), "source is a fluid cell", seed, (long)c, i);
          // byte offsets of the slots the kernels address (plane of opp(i) at the source)
          const uint64_t off = ((uint64_t)opp[i] * (uint64_t)plane_cells(L.nc) + (uint64_t)src) * 4u;
          expect(off < (1ull << 32), "32-bit byte offset", seed, (long)c, i);
          if (k > 0) rel_src[i] = c + (int64_t)L.rel.at((size_t)row * 8 + (k - 1)) - cv[i][0];
          else rel_src[i] = c - cv[i][0];
          true_src[i] = src;
        }
      }
      // neighbour x + c_i for the uniform-porosity flag
      int n[3];
      bool nout = false;
      for (int a = 0; a < 3; ++a) {
        n[a] = X[a] + cv[i][a];
        if (n[a] < 0 || n[a] >= dims[a]) {
          if (L.periodic[a]) n[a] = (n[a] + dims[a]) % dims[a];
          else nout = true;
        }
      }
      if (!nout) {
        const int64_t nb = (int64_t)n[0] + (int64_t)L.nx * ((int64_t)n[1] + (int64_t)L.ny * n[2]);
        if (!L.solid.at(nb) && phib.at(nb) != phib.at(b)) uni = false;
      }
    }
    expect(((lk & uni_bit) != 0) == uni, "uniform-neighbour-porosity flag", seed, (long)c, -1);
    const bool inr = !any_wall && !(L.periodic[0] && (x == 0 || x == L.nx - 1));
    if (inr_bit) expect(((lk & inr_bit) != 0) == inr, "interior flag", seed, (long)c, -1);
    if (inr) {
      // the interior path of a plain wave: c + rel[row][pair] - c_x for every direction
      for (int i = 1; i < NQ; ++i) {
        expect(rel_src[i] == true_src[i], "interior-path source from the row offsets", seed, (long)c, i);
        ++g_inr;
      }
    }
  }
}

// The per-wave row records as the wave-record kernel forms them (first row,
// a bit per lane that starts a new row), decoded as the step decodes them.
void check_wave_rows(const HostLayout& L, int seed) {
  const int64_t nrec = wave_records(L.nc);
  expect(nrec * 64 >= L.nc, "wave records cover the compact cells", seed, -1, -1);
  for (int64_t w = 0; w < nrec; ++w) {
    const int64_t c0 = w * 64;
    if (c0 >= L.nc) break;
    const uint32_t row0 = L.code.at(c0) >> L.xbits;
    uint64_t starts = 0;
    for (int l = 1; l < 64 && c0 + l < L.nc; ++l)
      if ((L.code.at(c0 + l) >> L.xbits) != (L.code.at(c0 + l - 1) >> L.xbits)) starts |= 1ull << l;
    for (int l = 0; l < 64 && c0 + l < L.nc; ++l) {
      const uint32_t row = row0 + (uint32_t)__builtin_popcountll(starts & ((2ull << l) - 2ull));
      expect(row == (L.code.at(c0 + l) >> L.xbits), "row decoded from the wave record", seed, (long)(c0 + l), -1);
    }
  }
}

void one_case(int seed) {
  std::mt19937_64 rng(1000 + seed);
  auto uni = [&](int lo, int hi) { return (int)std::uniform_int_distribution<int>(lo, hi)(rng); };
  auto u01 = [&]() { return std::uniform_real_distribution<double>(0.0, 1.0)(rng); };
  lbm_grid g{};
  g.nx = uni(1, 12); g.ny = uni(1, 12); g.nz = uni(1, 12);
  for (int a = 0; a < 3; ++a) g.periodic[a] = u01() < 0.4;
  const bool open = !g.periodic[0] && g.nx >= 2 && u01() < 0.6;
  const int outlet = open ? uni(0, 2) : 0;
  const bool inlet = open && u01() < 0.8;
  const size_t nbox = (size_t)g.nx * g.ny * g.nz;
  std::vector<uint8_t> solid(nbox), region(nbox);
  std::vector<float> phib(nbox);
  const double fs = 0.35 * u01();
  const bool varphi = u01() < 0.6;
  for (size_t b = 0; b < nbox; ++b) {
    solid[b] = u01() < fs;
    region[b] = u01() < 0.3;
    const int x = (int)(b % g.nx);
    const bool face = (inlet && x == 0) || (outlet && x == g.nx - 1);
    phib[b] = solid[b] ? 0.0f : (face || !varphi ? 1.0f : (float)(0.3 + 0.7 * (double)uni(0, 3) / 3.0));
  }
  solid[(size_t)uni(0, (int)nbox - 1)] = 0;  // at least one fluid cell
  HostLayout L;
  build_host_layout(L, g, solid.data(), region.data(), inlet, outlet);
  if (L.nf == 0) return;
  std::vector<uint32_t> l19;
  std::vector<uint64_t> l27;
  build_links(L, phib, l19);
  build_links27(L, phib, l27);
  int cv19[Q][3], cv27[q27::Q][3], pk19[Q], pk27[q27::Q], opp27[q27::Q];
  for (int i = 0; i < Q; ++i) { cv19[i][0] = CX[i]; cv19[i][1] = CY[i]; cv19[i][2] = CZ[i]; pk19[i] = PK[i]; }
  for (int i = 0; i < q27::Q; ++i) {
    cv27[i][0] = q27::CX[i]; cv27[i][1] = q27::CY[i]; cv27[i][2] = q27::CZ[i];
    pk27[i] = q27::pk(i); opp27[i] = q27::opp(i);
  }
  int opp19[Q];
  for (int i = 0; i < Q; ++i) opp19[i] = OPP[i];
  check_links<uint32_t, Q>(L, phib, l19, cv19, opp19, pk19, LK_DEAD, LK_UNI, LK_IN, LK_OUT, LK_UNK, XIN, XOUT, 5,
                           LK_INR, seed);
  check_wave_rows(L, seed);
  check_links<uint64_t, q27::Q>(L, phib, l27, cv27, opp27, pk27, q27::L_DEAD, q27::L_UNI, q27::L_IN, q27::L_OUT,
                                q27::L_UNK, q27::XIN, q27::XOUT, q27::NX, (uint64_t)0, seed);
}

}  // namespace

int main(int argc, char** argv) {
  const int n = argc > 1 ? std::atoi(argv[1]) : 400;
  for (int s = 0; s < n; ++s) one_case(s);
  std::printf("layout check: %d random boxes, %ld interior-path sources, %d failures\n", n, g_inr, g_fail);
  return (g_fail || g_inr == 0) ? 1 : 0;
}
