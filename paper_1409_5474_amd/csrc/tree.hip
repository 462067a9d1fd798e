// Barnes-Hut tree code on the GPU (the paper's collisionless method: section
// "Simulating collisionless systems with hierarchical domain-decomposition
// methods", subsection "Implementation"): every part runs on the device --
// Peano-Hilbert keys and the sort along the curve, an octree whose cells cut
// the curve into distinct pieces until a cell holds at most n_crit
// particles, monopole and quadrupole moments, groups of up to 64
// curve-consecutive particles (split while wider than g_max), the walk with
// a geometric opening criterion, and the force evaluation.
//
// Readings shared with the documentation of nb_tree_forces (nbody.h):
//  * box: lo = per-dimension minimum, side = 2^e >= (1 + 2^-10) * largest
//    extent, h = side 2^-21, integer coordinates floor((x - lo)/h) clamped
//  * keys: 63-bit Peano-Hilbert index (Skilling's construction), particles
//    sorted by (key, index) with a stable radix sort
//  * cell (l, p): the particles with key prefix p of 3l bits; split while it
//    holds more than n_crit particles (l < 21); cube corner from the first
//    particle's coordinates with the low 21-l bits cleared, side 2^(21-l) h
//  * a cell other than the root is accepted for a group when
//    theta^2 d^2 > side^2, d the distance between the group's bounding box
//    and the cube; an opened leaf's particles interact directly
//  * accepted cell: a = -M y s^-3/2 + Q y s^-5/2 - (5/2)(y.Qy) y s^-7/2,
//    phi = -M s^-1/2 - (y.Qy)/2 s^-5/2 with y = x - X, s = |y|^2 + eps2,
//    Q = sum m (3 d d^T - |d|^2 I) about the centre of mass X
//
// Structure on the chip: the build is level-synchronous and data-parallel
// -- one thread per particle or per cell, with the library's own stable
// radix sort and exclusive scans placing the outputs, so every array keeps
// curve order and the results are reproducible run to run.  The level
// bounds stay in device memory and the buffers are sized from bounds known
// up front, so nothing is read on the host until the forces are written and
// a whole evaluation can be captured in a graph.  The walk and the force evaluation are one kernel, as in the
// paper's GPU tree code: one wavefront per group walks the tree for its 64
// particles and evaluates accepted cells and opened leaves 64 at a time from
// LDS as it finds them, so no interaction list is written to memory.  The
// build and the walk are double precision; the force terms are double or
// mixed (float terms from double separations, summed in double per chunk)
// with the context's precision.  The opening test and the cube geometry are
// computed without fused multiply-adds, in the order stated above, so they
// match any implementation that rounds each operation.
#include <string>
#include <type_traits>
#include <vector>

#include "nb_internal.h"

namespace nb {
namespace {

constexpr int kBits = 21;
constexpr int kLevels = kBits + 1;  // cell levels 0 .. kBits
constexpr int kTB = 256;   // threads per block of the element-wise kernels
constexpr int kGS = 64;    // particles per group (one wavefront)

inline int blocks_for(int64_t n, int cap = 65535) {
  int64_t g = (n + kTB - 1) / kTB;
  return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}

struct Box {
  double lo[3];
  double side;
  double h;
};

// ---------------------------------------------------------------- box -----
__global__ __launch_bounds__(kTB) void k_bbox_partial(const double* __restrict__ pos, int64_t n,
                                                      double* __restrict__ part) {
  __shared__ double red[6][kTB];
  double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kTB)
    for (int c = 0; c < 3; ++c) {
      const double x = pos[3 * i + c];
      mn[c] = fmin(mn[c], x);
      mx[c] = fmax(mx[c], x);
    }
  for (int c = 0; c < 3; ++c) {
    red[c][threadIdx.x] = mn[c];
    red[3 + c][threadIdx.x] = mx[c];
  }
  __syncthreads();
  for (int o = kTB / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o)
      for (int c = 0; c < 3; ++c) {
        red[c][threadIdx.x] = fmin(red[c][threadIdx.x], red[c][threadIdx.x + o]);
        red[3 + c][threadIdx.x] = fmax(red[3 + c][threadIdx.x], red[3 + c][threadIdx.x + o]);
      }
    __syncthreads();
  }
  if (threadIdx.x < 6) part[6 * blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

__global__ __launch_bounds__(kTB) void k_bbox_final(const double* __restrict__ part, int nblk,
                                                    Box* __restrict__ box) {
  __shared__ double red[6][kTB];
  double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int b = threadIdx.x; b < nblk; b += kTB)
    for (int c = 0; c < 3; ++c) {
      mn[c] = fmin(mn[c], part[6 * b + c]);
      mx[c] = fmax(mx[c], part[6 * b + 3 + c]);
    }
  for (int c = 0; c < 3; ++c) {
    red[c][threadIdx.x] = mn[c];
    red[3 + c][threadIdx.x] = mx[c];
  }
  __syncthreads();
  for (int o = kTB / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o)
      for (int c = 0; c < 3; ++c) {
        red[c][threadIdx.x] = fmin(red[c][threadIdx.x], red[c][threadIdx.x + o]);
        red[3 + c][threadIdx.x] = fmax(red[3 + c][threadIdx.x], red[3 + c][threadIdx.x + o]);
      }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  double ext = 0.0;
  for (int c = 0; c < 3; ++c) ext = fmax(ext, red[3 + c][0] - red[c][0]);
  double side = 1.0;
  if (ext > 0.0) {
    int e = 0;
    (void)frexp(ext * (1.0 + 0x1p-10), &e);
    side = ldexp(1.0, e);
  }
  Box bx;
  for (int c = 0; c < 3; ++c) bx.lo[c] = red[c][0];
  bx.side = side;
  bx.h = ldexp(side, -kBits);
  *box = bx;
}

// --------------------------------------------------------------- keys -----
__device__ __forceinline__ void grid_of(const double* x, const Box& b, int32_t* q) {
  for (int c = 0; c < 3; ++c) {
    double v = floor((x[c] - b.lo[c]) / b.h);
    v = v < 0.0 ? 0.0 : (v > (double)((1 << kBits) - 1) ? (double)((1 << kBits) - 1) : v);
    q[c] = (int32_t)v;
  }
}

// Peano-Hilbert index of three 21-bit coordinates: plane by plane from the
// top, an axis whose bit is set flips the lower bits of axis 0, otherwise
// the two trade their lower bits; then Gray coding along the axes and the
// parity mask of the last axis; finally the bits interleaved from the top.
__device__ __forceinline__ uint64_t hilbert63(uint32_t a0, uint32_t a1, uint32_t a2) {
  uint32_t w[3] = {a0, a1, a2};
  for (uint32_t plane = 1u << (kBits - 1); plane > 1u; plane >>= 1) {
    const uint32_t low = plane - 1u;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (w[k] & plane) {
        w[0] ^= low;
      } else {
        const uint32_t d = (w[0] ^ w[k]) & low;
        w[0] ^= d;
        w[k] ^= d;
      }
    }
  }
  w[1] ^= w[0];
  w[2] ^= w[1];
  uint32_t mask = 0;
  for (uint32_t plane = 1u << (kBits - 1); plane > 1u; plane >>= 1)
    if (w[2] & plane) mask ^= plane - 1u;
  w[0] ^= mask; w[1] ^= mask; w[2] ^= mask;
  uint64_t key = 0;
  for (int b = kBits - 1; b >= 0; --b)
#pragma unroll
    for (int k = 0; k < 3; ++k) key = (key << 1) | ((w[k] >> b) & 1u);
  return key;
}

__global__ __launch_bounds__(kTB) void k_keys(const double* __restrict__ pos, int64_t n, const Box* __restrict__ box,
                                              uint64_t* __restrict__ keys, int32_t* __restrict__ idx) {
  const Box b = *box;
  for (int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kTB) {
    int32_t q[3];
    grid_of(pos + 3 * i, b, q);
    keys[i] = hilbert63((uint32_t)q[0], (uint32_t)q[1], (uint32_t)q[2]);
    idx[i] = (int32_t)i;
  }
}

__global__ __launch_bounds__(kTB) void k_gather(const double* __restrict__ pos, const double* __restrict__ mass,
                                                const int32_t* __restrict__ idx, int64_t n,
                                                const Box* __restrict__ box, double* __restrict__ pos_s,
                                                double* __restrict__ mass_s, int32_t* __restrict__ ijk_s) {
  const Box b = *box;
  for (int64_t k = (int64_t)blockIdx.x * kTB + threadIdx.x; k < n; k += (int64_t)gridDim.x * kTB) {
    const int64_t i = idx[k];
    for (int c = 0; c < 3; ++c) pos_s[3 * k + c] = pos[3 * i + c];
    mass_s[k] = mass[i];
    grid_of(pos + 3 * i, b, ijk_s + 3 * k);
  }
}

// --------------------------------------------------------------- tree -----
__device__ __forceinline__ void set_geometry(TreeCell& c, const int32_t* ijk_s, const Box& b) {
#pragma clang fp contract(off)
  const int shift = kBits - c.level;
  for (int k = 0; k < 3; ++k) {
    const int64_t ci = ((int64_t)ijk_s[3 * c.begin + k] >> shift) << shift;
    c.corner[k] = b.lo[k] + (double)ci * b.h;
  }
  c.side = ldexp(b.h, shift);
}

// The root, and the level table: the cells of level l are [lvl[l], lvl[l+1])
// (kept in device memory, so no count goes to the host while the tree grows).
__global__ void k_root(TreeCell* __restrict__ cells, int32_t n, const int32_t* __restrict__ ijk_s,
                       const Box* __restrict__ box, int32_t* __restrict__ lvl) {
  if (blockIdx.x != 0) return;
  for (int l = threadIdx.x; l < kLevels + 1; l += blockDim.x) lvl[l] = l == 0 ? 0 : 1;
  if (threadIdx.x != 0) return;
  TreeCell c{};
  c.begin = 0; c.end = n; c.child0 = -1; c.nchild = 0; c.level = 0;
  set_geometry(c, ijk_s, *box);
  cells[0] = c;
}

// first position in [lo, hi) whose key is >= bound
__device__ __forceinline__ int32_t lower_bound_key(const uint64_t* keys, int32_t lo, int32_t hi, uint64_t bound) {
  while (lo < hi) {
    const int32_t mid = lo + (hi - lo) / 2;
    if (keys[mid] < bound) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// The child boundaries of every cell that splits, kept in `ends` [ncell][8]
// for the write pass: eight consecutive lanes per cell, lane k finds where
// child k ends (a binary search over the cell's keys; child k of a cell at
// level l covers the keys [(p<<3|k) << s, (p<<3|k)+1 << s), s = 3(20 - l),
// and the last child ends with the cell), and the cell's count of non-empty
// children is summed over the eight lanes.
__global__ __launch_bounds__(kTB) void k_count_children(const TreeCell* __restrict__ all_cells,
                                                        const int32_t* __restrict__ lvl, int l,
                                                        const uint64_t* __restrict__ keys, int n_crit,
                                                        int32_t* __restrict__ cnt, int32_t* __restrict__ ends) {
  const TreeCell* cells = all_cells + lvl[l];
  const int32_t ncell = lvl[l + 1] - lvl[l];
  const int64_t total = 8 * (int64_t)ncell;  // whole groups of eight lanes
  for (int64_t t = (int64_t)blockIdx.x * kTB + threadIdx.x; t < total; t += (int64_t)gridDim.x * kTB) {
    const int32_t i = (int32_t)(t >> 3);
    const int k = (int)(t & 7);
    const TreeCell& c = cells[i];
    const bool split = c.end - c.begin > n_crit && c.level < kBits;
    int32_t e = c.end;
    if (split && k < 7) {
      const int sh = 3 * (kBits - c.level - 1);
      const uint64_t prefix = keys[c.begin] >> (sh + 3);
      e = lower_bound_key(keys, c.begin, c.end, ((prefix << 3) | (uint64_t)(k + 1)) << sh);
    }
    const int32_t prev = __shfl_up(e, 1, 8);
    const int32_t b = k == 0 ? c.begin : prev;
    int m = (split && e > b) ? 1 : 0;
    m += __shfl_xor(m, 1, 8);
    m += __shfl_xor(m, 2, 8);
    m += __shfl_xor(m, 4, 8);
    if (split) ends[t] = e;
    if (k == 0) cnt[i] = m;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) cnt[ncell] = 0;
}

__global__ __launch_bounds__(kTB) void k_write_children(TreeCell* __restrict__ cells, int32_t* __restrict__ lvl, int l,
                                                        const int32_t* __restrict__ ends,
                                                        const int32_t* __restrict__ ijk_s,
                                                        const Box* __restrict__ box, int n_crit,
                                                        const int32_t* __restrict__ off) {
  const int32_t first = lvl[l], next = lvl[l + 1], ncell = next - first;
  const Box bx = *box;
  // the next level's cells follow this one's; off[ncell] is their number
  if (blockIdx.x == 0 && threadIdx.x == 0) lvl[l + 2] = next + off[ncell];
  for (int32_t i = blockIdx.x * kTB + threadIdx.x; i < ncell; i += gridDim.x * kTB) {
    TreeCell& c = cells[first + i];
    if (!(c.end - c.begin > n_crit && c.level < kBits)) {
      c.child0 = -1;
      c.nchild = 0;
      continue;
    }
    const int32_t base = next + off[i];
    int32_t b = c.begin, m = 0;
    for (int k = 0; k < 8; ++k) {
      const int32_t e = ends[8 * (int64_t)i + k];
      if (e > b) {
        TreeCell ch{};
        ch.begin = b; ch.end = e; ch.child0 = -1; ch.nchild = 0; ch.level = c.level + 1;
        set_geometry(ch, ijk_s, bx);
        cells[base + m] = ch;
        ++m;
      }
      b = e;
    }
    c.child0 = base;
    c.nchild = m;
  }
}

// Moments: leaves from their particles, internal cells from their children.
__global__ __launch_bounds__(kTB) void k_moments(TreeCell* __restrict__ cells, const int32_t* __restrict__ lvl, int l,
                                                 const double* __restrict__ pos_s, const double* __restrict__ mass_s) {
  const int32_t first = lvl[l], ncell = lvl[l + 1] - lvl[l];
  for (int32_t i = blockIdx.x * kTB + threadIdx.x; i < ncell; i += gridDim.x * kTB) {
    TreeCell& c = cells[first + i];
    double M = 0.0, S[3] = {0.0, 0.0, 0.0}, Q[6] = {0, 0, 0, 0, 0, 0}, X[3];
    if (c.nchild == 0) {
      for (int32_t j = c.begin; j < c.end; ++j) {
        const double m = mass_s[j];
        M += m;
        for (int k = 0; k < 3; ++k) S[k] += m * pos_s[3 * j + k];
      }
      for (int k = 0; k < 3; ++k) X[k] = M > 0.0 ? S[k] / M : c.corner[k] + 0.5 * c.side;
      for (int32_t j = c.begin; j < c.end; ++j) {
        const double m = mass_s[j];
        const double d0 = pos_s[3 * j] - X[0], d1 = pos_s[3 * j + 1] - X[1], d2 = pos_s[3 * j + 2] - X[2];
        const double dd = d0 * d0 + d1 * d1 + d2 * d2;
        Q[0] += m * (3.0 * (d0 * d0) - dd);
        Q[1] += m * (3.0 * (d1 * d1) - dd);
        Q[2] += m * (3.0 * (d2 * d2) - dd);
        Q[3] += m * (3.0 * (d0 * d1));
        Q[4] += m * (3.0 * (d0 * d2));
        Q[5] += m * (3.0 * (d1 * d2));
      }
    } else {
      for (int32_t k = 0; k < c.nchild; ++k) {
        const TreeCell& ch = cells[c.child0 + k];
        M += ch.M;
        for (int q = 0; q < 3; ++q) S[q] += ch.M * ch.X[q];
      }
      for (int k = 0; k < 3; ++k) X[k] = M > 0.0 ? S[k] / M : c.corner[k] + 0.5 * c.side;
      for (int32_t k = 0; k < c.nchild; ++k) {
        const TreeCell& ch = cells[c.child0 + k];
        const double e0 = ch.X[0] - X[0], e1 = ch.X[1] - X[1], e2 = ch.X[2] - X[2];
        const double ee = e0 * e0 + e1 * e1 + e2 * e2;
        const double m = ch.M;
        Q[0] += ch.Q[0] + m * (3.0 * (e0 * e0) - ee);
        Q[1] += ch.Q[1] + m * (3.0 * (e1 * e1) - ee);
        Q[2] += ch.Q[2] + m * (3.0 * (e2 * e2) - ee);
        Q[3] += ch.Q[3] + m * (3.0 * (e0 * e1));
        Q[4] += ch.Q[4] + m * (3.0 * (e0 * e2));
        Q[5] += ch.Q[5] + m * (3.0 * (e1 * e2));
      }
    }
    c.M = M;
    for (int k = 0; k < 3; ++k) c.X[k] = X[k];
    for (int k = 0; k < 6; ++k) c.Q[k] = Q[k];
  }
}

// ------------------------------------------------------------- groups -----
__device__ __forceinline__ double extent(const double* pos_s, int32_t b, int32_t e) {
  double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int32_t j = b; j < e; ++j)
    for (int k = 0; k < 3; ++k) {
      mn[k] = fmin(mn[k], pos_s[3 * j + k]);
      mx[k] = fmax(mx[k], pos_s[3 * j + k]);
    }
  return fmax(mx[0] - mn[0], fmax(mx[1] - mn[1], mx[2] - mn[2]));
}

// number of set bits of `mask` below this lane
__device__ __forceinline__ int lane_rank(uint64_t mask) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Groups of one curve chunk of up to 64 particles: the chunk is halved
// (first half ceil(n/2)) while a piece holding more than one particle is
// wider than g_max, first half first.  An explicit stack replaces the
// recursion; a chunk of 64 is halved at most six times, so seven entries
// suffice.  Returns the number of groups; writes them when `gb` is set.
__device__ __forceinline__ int32_t split_chunk(const double* __restrict__ pos_s, int32_t b0, int32_t e0,
                                               double g_max, int32_t* __restrict__ gb, int32_t* __restrict__ ge) {
  int32_t sb[8], se[8];
  int sp = 1;
  sb[0] = b0;
  se[0] = e0;
  int32_t cnt = 0;
  while (sp > 0) {
    --sp;
    const int32_t b = sb[sp], e = se[sp];
    if (e - b > 1 && sp + 2 <= 8 && extent(pos_s, b, e) > g_max) {
      const int32_t m = b + (e - b + 1) / 2;
      sb[sp] = m; se[sp] = e; ++sp;
      sb[sp] = b; se[sp] = m; ++sp;
    } else {
      if (gb) {
        gb[cnt] = b;
        ge[cnt] = e;
      }
      ++cnt;
    }
  }
  return cnt;
}

// One wavefront per chunk.  A full chunk of 64 is only ever cut at aligned
// halves, and a piece that fits (extent <= g_max) has pieces that fit, so
// the group holding particle j is the largest aligned piece around j that
// fits (a single particle always does): lane j reduces the minimum and
// maximum position over the aligned pieces of 2, 4, ..., 64 around it by
// butterfly shuffles and keeps the largest size that fits.  The last,
// shorter chunk takes the recursion above on lane 0.  WRITE = false counts
// the groups per chunk, WRITE = true writes them at their offsets.
template <bool WRITE>
__global__ __launch_bounds__(kTB) void k_groups(int32_t n, int32_t nchunk, const double* __restrict__ pos_s,
                                                const Box* __restrict__ box, double g_frac,
                                                int32_t* __restrict__ cnt, const int32_t* __restrict__ off,
                                                int32_t* __restrict__ gb, int32_t* __restrict__ ge,
                                                int32_t* __restrict__ ng) {
  const double g_max = g_frac > 0.0 ? g_frac * box->side : INFINITY;
  const int lane = threadIdx.x & (kGS - 1);
  const int64_t wave = ((int64_t)blockIdx.x * kTB + threadIdx.x) / kGS;
  const int64_t nwaves = (int64_t)gridDim.x * kTB / kGS;
  for (int64_t c = wave; c < nchunk; c += nwaves) {
    const int32_t b = (int32_t)c * kGS, e = b + kGS < n ? b + kGS : n;
    if (e - b < kGS) {
      if (lane == 0) {
        if (WRITE) split_chunk(pos_s, b, e, g_max, gb + off[c], ge + off[c]);
        else cnt[c] = split_chunk(pos_s, b, e, g_max, nullptr, nullptr);
      }
      continue;
    }
    const int32_t j = b + lane;
    double mn[3], mx[3];
    for (int k = 0; k < 3; ++k) mn[k] = mx[k] = pos_s[3 * j + k];
    int size = 1;
    for (int h = 1; h < kGS; h <<= 1) {
      for (int k = 0; k < 3; ++k) {
        mn[k] = fmin(mn[k], __shfl_xor(mn[k], h, kGS));
        mx[k] = fmax(mx[k], __shfl_xor(mx[k], h, kGS));
      }
      const double ext = fmax(mx[0] - mn[0], fmax(mx[1] - mn[1], mx[2] - mn[2]));
      if (size == h && !(ext > g_max)) size = 2 * h;
    }
    const bool start = (lane & (size - 1)) == 0;
    const uint64_t starts = __ballot(start);
    if (WRITE) {
      if (start) {
        const int32_t o = off[c] + lane_rank(starts);
        gb[o] = j;
        ge[o] = j + size;
      }
    } else if (lane == 0) {
      cnt[c] = __popcll(starts);
    }
  }
  if (WRITE && blockIdx.x == 0 && threadIdx.x == 0) *ng = off[nchunk - 1] + cnt[nchunk - 1];
}

__global__ __launch_bounds__(kTB) void k_group_box(const int32_t* __restrict__ gb, const int32_t* __restrict__ ge,
                                                   const int32_t* __restrict__ ng_dev, const double* __restrict__ pos_s,
                                                   double* __restrict__ gbox) {
  const int32_t ng = *ng_dev;
  for (int32_t g = blockIdx.x * kTB + threadIdx.x; g < ng; g += gridDim.x * kTB) {
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int32_t j = gb[g]; j < ge[g]; ++j)
      for (int k = 0; k < 3; ++k) {
        mn[k] = fmin(mn[k], pos_s[3 * j + k]);
        mx[k] = fmax(mx[k], pos_s[3 * j + k]);
      }
    for (int k = 0; k < 3; ++k) {
      gbox[6 * g + k] = mn[k];
      gbox[6 * g + 3 + k] = mx[k];
    }
  }
}

// ------------------------------------------------- walk and forces -----
// One kernel does the walk and the force evaluation, as the paper's GPU
// tree code does: a wavefront takes a group (its lanes are the group's
// particles), walks the tree for the whole group, and evaluates the accepted
// cells and the particles of opened leaves as soon as 64 of them are
// pending.  No interaction list goes to memory; the only memory beyond the
// tree is a per-wavefront stack of cells still to be tested.
//
// Walk step: pop up to 64 cells from the top of the stack, one per lane;
// each lane tests its cell and the wavefront appends accepted cells and
// opened leaves to two LDS lists (ballot + rank) and pushes the children of
// opened internal cells, in lane order, onto the stack (wave prefix sum).
// Bound on the stack: the pushes keep it ordered by level from bottom to
// top (lane order is stack order, children sit one level below their
// parents, and what is left after a pop is no deeper than what was popped).
// Level-l entries are pushed only by a pop that took level-(l-1) entries,
// and such a pop took every entry of level >= l, which lie above them; so
// the level-l entries on the stack always come from one push of at most
// 8 x 64 entries, and the stack holds at most 8 x 64 x 21 entries (levels
// 1 to 21).  It also never holds more entries than there are cells, since
// a cell is pushed at most once per group.  The kernel still checks every
// push against the capacity and reports an overflow instead of writing
// past it.
constexpr int kStackCap = 8 * kGS * kBits;

__device__ __forceinline__ bool accepted(const TreeCell& c, const double* gbox, double theta) {
#pragma clang fp contract(off)
  double d2 = 0.0;
  for (int k = 0; k < 3; ++k) {
    const double a = c.corner[k] - gbox[3 + k];
    const double b = gbox[k] - (c.corner[k] + c.side);
    double gap = a > b ? a : b;
    gap = gap > 0.0 ? gap : 0.0;
    d2 = k == 0 ? gap * gap : d2 + gap * gap;
  }
  return theta * theta * d2 > c.side * c.side;
}

// s^{-1/2}: v_rsq_f64 (about 2^-24 accurate) refined by one third-order
// Newton step y (1 + e/2 + 3e^2/8), e = 1 - s y^2, to double rounding.
__device__ __forceinline__ double rsqrt_tree(double s) {
  const double y = __builtin_amdgcn_rsq(s);
  const double e = fma(-(s * y), y, 1.0);
  return fma(y, e * fma(e, 0.375, 0.5), y);
}


__device__ __forceinline__ int wave_inclusive_sum(int v, int lane) {
  for (int d = 1; d < kGS; d <<= 1) {
    const int t = __shfl_up(v, d, kGS);
    if (lane >= d) v += t;
  }
  return v;
}

struct CellLite {
  double M, X[3], Q[6];
};
// Mixed precision: the separation from a cell's centre of mass or from a
// particle is formed in double and rounded to float, the rest of the term
// is float; the float sums of one staged chunk (at most 64 cells or 64
// particles) are added into double accumulators.  The walk, and so the
// interaction set, is the double one.
struct CellLiteF {
  double X[3];
  float M, Q[6], pad;
};

// LDS of one wavefront: the staged cells and the staged leaf particles are
// never live at the same time and share their storage.
template <bool MIXED>
struct WalkLds {
  using Cell = typename std::conditional<MIXED, CellLiteF, CellLite>::type;
  struct Parts {
    double px[kGS], py[kGS], pz[kGS], pm[kGS];
    int32_t pj[kGS];
  };
  union {
    Cell tile[kGS];
    Parts p;
  };
  int32_t acc_list[2 * kGS];
  int32_t leaf_list[2 * kGS];
  int32_t leaf_begin[kGS];
  int32_t leaf_pre[kGS + 1];
};

struct Accum {
  double a0, a1, a2, ph;
};

// The first `cnt` (<= 64) accepted cells of the list: each lane stages one
// cell, then every lane adds all of them to its particle.
template <bool MIXED>
__device__ __forceinline__ void eval_cells(WalkLds<MIXED>& L, int cnt, const TreeCell* __restrict__ cells,
                                           double x0, double x1, double x2, double eps2, Accum& A, int lane) {
  if (lane < cnt) {
    const TreeCell& c = cells[L.acc_list[lane]];
    if constexpr (MIXED) {
      CellLiteF cl;
      cl.M = (float)c.M;
      for (int q = 0; q < 3; ++q) cl.X[q] = c.X[q];
      for (int q = 0; q < 6; ++q) cl.Q[q] = (float)c.Q[q];
      cl.pad = 0.0f;
      L.tile[lane] = cl;
    } else {
      CellLite cl;
      cl.M = c.M;
      for (int q = 0; q < 3; ++q) cl.X[q] = c.X[q];
      for (int q = 0; q < 6; ++q) cl.Q[q] = c.Q[q];
      L.tile[lane] = cl;
    }
  }
  __syncthreads();
  if constexpr (MIXED) {
    const float e2 = (float)eps2;
    float f0 = 0.0f, f1 = 0.0f, f2 = 0.0f, fp = 0.0f;
    for (int t = 0; t < cnt; ++t) {
      const CellLiteF& c = L.tile[t];
      const float y0 = (float)(x0 - c.X[0]), y1 = (float)(x1 - c.X[1]), y2 = (float)(x2 - c.X[2]);
      const float s = fmaf(y2, y2, fmaf(y1, y1, fmaf(y0, y0, e2)));
      const float q = __builtin_amdgcn_rsqf(s);
      const float q2 = q * q;
      const float q3 = q2 * q, q5 = q3 * q2;
      const float Qy0 = c.Q[0] * y0 + c.Q[3] * y1 + c.Q[4] * y2;
      const float Qy1 = c.Q[3] * y0 + c.Q[1] * y1 + c.Q[5] * y2;
      const float Qy2 = c.Q[4] * y0 + c.Q[5] * y1 + c.Q[2] * y2;
      const float w = (y0 * Qy0 + y1 * Qy1 + y2 * Qy2) * q5;  // (y.Qy) s^-5/2
      const float f = fmaf(-2.5f * w, q2, -c.M * q3);         // -M s^-3/2 - (5/2)(y.Qy) s^-7/2
      f0 = fmaf(Qy0, q5, fmaf(f, y0, f0));
      f1 = fmaf(Qy1, q5, fmaf(f, y1, f1));
      f2 = fmaf(Qy2, q5, fmaf(f, y2, f2));
      fp = fmaf(-0.5f, w, fmaf(-c.M, q, fp));
    }
    A.a0 += (double)f0; A.a1 += (double)f1; A.a2 += (double)f2; A.ph += (double)fp;
  } else {
    for (int t = 0; t < cnt; ++t) {
      const CellLite& c = L.tile[t];
      const double y0 = x0 - c.X[0], y1 = x1 - c.X[1], y2 = x2 - c.X[2];
      const double s = fma(y2, y2, fma(y1, y1, fma(y0, y0, eps2)));
      const double q = rsqrt_tree(s);
      const double q2 = q * q;
      const double q3 = q2 * q, q5 = q3 * q2;
      const double Qy0 = c.Q[0] * y0 + c.Q[3] * y1 + c.Q[4] * y2;
      const double Qy1 = c.Q[3] * y0 + c.Q[1] * y1 + c.Q[5] * y2;
      const double Qy2 = c.Q[4] * y0 + c.Q[5] * y1 + c.Q[2] * y2;
      const double w = (y0 * Qy0 + y1 * Qy1 + y2 * Qy2) * q5;  // (y.Qy) s^-5/2
      const double f = fma(-2.5 * w, q2, -c.M * q3);          // -M s^-3/2 - (5/2)(y.Qy) s^-7/2
      A.a0 = fma(Qy0, q5, fma(f, y0, A.a0));
      A.a1 = fma(Qy1, q5, fma(f, y1, A.a1));
      A.a2 = fma(Qy2, q5, fma(f, y2, A.a2));
      A.ph = fma(-0.5, w, fma(-c.M, q, A.ph));
    }
  }
  __syncthreads();
}

// The particles of the first `cnt` (<= 64) opened leaves of the list, 64 at
// a time: lane p stages particle p of the chunk (found by a binary search
// over the leaves' prefix sums), then every lane adds the chunk's pair terms
// to its particle, skipping itself and coincident particles.
template <bool MIXED>
__device__ __forceinline__ void eval_leaves(WalkLds<MIXED>& L, int cnt, const TreeCell* __restrict__ cells,
                                            const double* __restrict__ pos_s, const double* __restrict__ mass_s,
                                            int32_t i, double x0, double x1, double x2, double eps2, Accum& A,
                                            int lane) {
  int size = 0, begin = 0;
  if (lane < cnt) {
    const TreeCell& c = cells[L.leaf_list[lane]];
    begin = c.begin;
    size = c.end - c.begin;
  }
  const int incl = wave_inclusive_sum(size, lane);
  const int total = __shfl(incl, kGS - 1, kGS);
  L.leaf_begin[lane] = begin;
  L.leaf_pre[lane + 1] = incl;
  if (lane == 0) L.leaf_pre[0] = 0;
  __syncthreads();
  for (int base = 0; base < total; base += kGS) {
    const int f = base + lane;
    if (f < total) {
      // the leaf k < cnt with leaf_pre[k] <= f < leaf_pre[k + 1]
      int lo = 0, hi = cnt - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (L.leaf_pre[mid] <= f) lo = mid;
        else hi = mid - 1;
      }
      const int32_t j = L.leaf_begin[lo] + (f - L.leaf_pre[lo]);
      L.p.px[lane] = pos_s[3 * j];
      L.p.py[lane] = pos_s[3 * j + 1];
      L.p.pz[lane] = pos_s[3 * j + 2];
      L.p.pm[lane] = mass_s[j];
      L.p.pj[lane] = j;
    }
    __syncthreads();
    const int m = total - base < kGS ? total - base : kGS;
    if constexpr (MIXED) {
      const float e2 = (float)eps2;
      float f0 = 0.0f, f1 = 0.0f, f2 = 0.0f, fp = 0.0f;
#pragma unroll 4
      for (int t = 0; t < m; ++t) {
        const float r0 = (float)(L.p.px[t] - x0), r1 = (float)(L.p.py[t] - x1), r2 = (float)(L.p.pz[t] - x2);
        const float s = fmaf(r2, r2, fmaf(r1, r1, fmaf(r0, r0, e2)));
        const bool keep = L.p.pj[t] != i && s > 0.0f;
        const float q = keep ? __builtin_amdgcn_rsqf(s) : 0.0f;
        const float mq = (float)L.p.pm[t] * q;
        const float mq3 = mq * q * q;
        f0 += mq3 * r0;
        f1 += mq3 * r1;
        f2 += mq3 * r2;
        fp -= mq;
      }
      A.a0 += (double)f0; A.a1 += (double)f1; A.a2 += (double)f2; A.ph += (double)fp;
    } else {
#pragma unroll 4
      for (int t = 0; t < m; ++t) {
        const double r0 = L.p.px[t] - x0, r1 = L.p.py[t] - x1, r2 = L.p.pz[t] - x2;
        const double s = fma(r2, r2, fma(r1, r1, fma(r0, r0, eps2)));
        const bool keep = L.p.pj[t] != i && s > 0.0;
        const double q = keep ? rsqrt_tree(s) : 0.0;
        const double mq = L.p.pm[t] * q;
        const double mq3 = mq * q * q;
        A.a0 += mq3 * r0;
        A.a1 += mq3 * r1;
        A.a2 += mq3 * r2;
        A.ph -= mq;
      }
    }
    __syncthreads();
  }
}

// drop the first 64 entries of a list of n (64 <= n < 128)
__device__ __forceinline__ void shift_list(int32_t* list, int n, int lane) {
  const int32_t v = lane + kGS < n ? list[lane + kGS] : 0;
  __syncthreads();
  if (lane + kGS < n) list[lane] = v;
  __syncthreads();
}

// Waves per SIMD asked of the register allocator.
#ifndef NB_TREE_WAVES
#define NB_TREE_WAVES 1
#endif

// counters[0]: next group, [1]: accepted (group, cell) pairs, [2]: opened
// (group, leaf) pairs, [3]: stack overflow flag
template <bool MIXED>
__global__ __launch_bounds__(kGS, NB_TREE_WAVES) void k_tree_walk_forces(const int32_t* __restrict__ gb,
                                                          const int32_t* __restrict__ ge,
                                                          const int32_t* __restrict__ ngroups_dev,
                                                          const double* __restrict__ gbox,
                                                          const TreeCell* __restrict__ cells, double theta,
                                                          const double* __restrict__ pos_s,
                                                          const double* __restrict__ mass_s, double eps2,
                                                          const int32_t* __restrict__ idx_s,
                                                          int32_t* __restrict__ stack_all, int32_t stack_cap,
                                                          unsigned long long* __restrict__ counters,
                                                          unsigned int* __restrict__ err,
                                                          double* __restrict__ acc, double* __restrict__ pot) {
  __shared__ WalkLds<MIXED> L;
  const int lane = threadIdx.x;
  const int32_t ngroups = *ngroups_dev;
  int32_t* stack = stack_all + (int64_t)blockIdx.x * stack_cap;
  const int32_t root_child0 = cells[0].child0, root_nchild = cells[0].nchild;
  for (;;) {
    int32_t g = 0;
    if (lane == 0) g = (int32_t)atomicAdd(&counters[0], 1ull);
    g = __shfl(g, 0, kGS);
    if (g >= ngroups) break;
    const int32_t b = gb[g], e = ge[g];
    const int32_t i = b + lane;
    const bool valid = i < e;
    const int32_t ir = valid ? i : b;
    const double x0 = pos_s[3 * ir], x1 = pos_s[3 * ir + 1], x2 = pos_s[3 * ir + 2];
    double box[6];
    for (int k = 0; k < 6; ++k) box[k] = gbox[6 * g + k];
    Accum A{0.0, 0.0, 0.0, 0.0};
    // the root is never accepted: the walk starts from its children, or
    // opens it when it is a leaf
    int sp = 0, n_acc = 0, n_leaf = 0;
    unsigned long long tot_acc = 0, tot_leaf = 0;
    bool overflow = false;
    if (root_nchild > 0) {
      if (lane < root_nchild) stack[lane] = root_child0 + lane;
      sp = root_nchild;
    } else {
      if (lane == 0) L.leaf_list[0] = 0;
      n_leaf = 1;
      tot_leaf = 1;
    }
    __syncthreads();
    while (sp > 0) {
      const int k = sp < kGS ? sp : kGS;
      const int base = sp - k;
      int kind = 3, nch = 0, ch0 = 0;
      int32_t cid = 0;
      if (lane < k) {
        cid = stack[base + lane];
        const TreeCell& c = cells[cid];
        if (accepted(c, box, theta)) {
          kind = 0;
        } else if (c.nchild == 0) {
          kind = 1;
        } else {
          kind = 2;
          nch = c.nchild;
          ch0 = c.child0;
        }
      }
      sp = base;
      const uint64_t ma = __ballot(kind == 0), ml = __ballot(kind == 1);
      if (kind == 0) L.acc_list[n_acc + lane_rank(ma)] = cid;
      if (kind == 1) L.leaf_list[n_leaf + lane_rank(ml)] = cid;
      n_acc += __popcll(ma);
      n_leaf += __popcll(ml);
      tot_acc += __popcll(ma);
      tot_leaf += __popcll(ml);
      const int incl = wave_inclusive_sum(nch, lane);
      const int pushed = __shfl(incl, kGS - 1, kGS);
      if (sp + pushed > stack_cap) {
        overflow = true;
        break;
      }
      for (int t = 0; t < nch; ++t) stack[sp + incl - nch + t] = ch0 + t;
      sp += pushed;
      __syncthreads();
      if (n_acc >= kGS) {
        eval_cells<MIXED>(L, kGS, cells, x0, x1, x2, eps2, A, lane);
        shift_list(L.acc_list, n_acc, lane);
        n_acc -= kGS;
      }
      if (n_leaf >= kGS) {
        eval_leaves<MIXED>(L, kGS, cells, pos_s, mass_s, i, x0, x1, x2, eps2, A, lane);
        shift_list(L.leaf_list, n_leaf, lane);
        n_leaf -= kGS;
      }
    }
    __syncthreads();
    if (!overflow) {
      if (n_acc > 0) eval_cells<MIXED>(L, n_acc, cells, x0, x1, x2, eps2, A, lane);
      if (n_leaf > 0) eval_leaves<MIXED>(L, n_leaf, cells, pos_s, mass_s, i, x0, x1, x2, eps2, A, lane);
      if (valid) {
        const int32_t o = idx_s[i];
        acc[3 * o] = A.a0;
        acc[3 * o + 1] = A.a1;
        acc[3 * o + 2] = A.a2;
        pot[o] = A.ph;
      }
    }
    if (lane == 0) {
      atomicAdd(&counters[1], tot_acc);
      atomicAdd(&counters[2], tot_leaf);
      if (overflow) {
        atomicOr(&counters[3], 1ull);
        if (err) atomicOr(err, kErrTreeStack);
      }
    }
    __syncthreads();
  }
}

__global__ void k_zero_u64(unsigned long long* p, int n) {
  if (blockIdx.x == 0 && (int)threadIdx.x < n) p[threadIdx.x] = 0ull;
}

// ---------------------------------------------------------------- scans -----
// Exclusive prefix sum of n int32 counts by one workgroup (out may be in), in
// rounds of kScanThreads x kScanPer consecutive entries: each thread loads
// kScanPer consecutive counts, the thread sums are scanned within each
// wavefront by shuffles and across the wavefronts through LDS (one barrier
// per round: the wavefront totals alternate between two buffers, and a
// wavefront can only overwrite a buffer after every wavefront has passed the
// next round's barrier, i.e. finished reading it), and each thread writes its
// entries' running sums.  Entries are read before they are written, by the
// same thread, so out may be in.  n is n_host, or, when lvl is set, the cell
// count of level l plus one (the extra zero count makes the last entry the
// level's total).  Every sum counts cells or particles, so it stays below
// 2^31.
constexpr int kScanThreads = 1024;
constexpr int kScanPer = 16;

__global__ __launch_bounds__(kScanThreads) void k_exscan(const int32_t* in, int32_t* out, int64_t n_host,
                                                         const int32_t* __restrict__ lvl, int l) {
  constexpr int W = kScanThreads / 64;
  __shared__ int32_t wsum[2][W];
  const int64_t n = lvl ? (int64_t)(lvl[l + 1] - lvl[l]) + 1 : n_host;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  int32_t carry = 0;
  int buf = 0;
  for (int64_t base = 0; base < n; base += (int64_t)kScanThreads * kScanPer) {
    const int64_t b = base + (int64_t)t * kScanPer;
    int32_t v[kScanPer];
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) v[j] = b + j < n ? in[b + j] : 0;
    int32_t sum = 0;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) sum += v[j];
    int32_t x = sum;  // inclusive scan of the thread sums over the wavefront
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int32_t y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) wsum[buf][wave] = x;
    __syncthreads();
    int32_t before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const int32_t ws = wsum[buf][w];
      before += w < wave ? ws : 0;
      total += ws;
    }
    int32_t run = carry + before + x - sum;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
      if (b + j < n) out[b + j] = run;
      run += v[j];
    }
    carry += total;
    buf ^= 1;
  }
}

// ----------------------------------------------------------- radix sort -----
// Stable least-significant-digit radix sort of (key, row) pairs, 8 bits per
// pass.  A pass: each tile of kRsTile keys counts its digits (k_rs_hist);
// the prefix of each digit's row of tile counts (k_rs_rowscan, one block
// per digit) plus the prefix of the digit totals gives every (digit, tile)
// its first output slot; each tile then writes its keys there
// (k_rs_scatter), a key's place among the equal digits of its tile being
// the number of such keys before it.  Within a tile, wavefront w takes the
// w-th quarter in rounds of 64 consecutive keys; the lanes of a round that
// share a digit find each other with eight ballots (one per digit bit), and
// a per-wavefront count of each digit carries over between rounds, so the
// order among equal digits is the input order.
constexpr int kRsBits = 8;
constexpr int kRsBuckets = 1 << kRsBits;
constexpr int kRsThreads = 256;
constexpr int kRsRounds = 8;                                 // rounds of 64 keys per wavefront
constexpr int kRsTile = (kRsThreads / 64) * 64 * kRsRounds;  // 2048 keys per tile
static_assert(kRsBuckets == kRsThreads, "one thread per digit in the tile tables");

__global__ __launch_bounds__(kRsThreads) void k_rs_hist(const uint64_t* __restrict__ keys, int32_t n, int shift,
                                                        int32_t* __restrict__ hist, int32_t ntile) {
  __shared__ int32_t h[kRsBuckets];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRsTile;
  for (int r = 0; r < kRsTile / kRsThreads; ++r) {
    const int64_t i = base + r * kRsThreads + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & (kRsBuckets - 1)], 1);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * ntile + blockIdx.x] = h[threadIdx.x];
}

// Per digit (block d): the exclusive prefix of its row of tile counts, in
// place (the tile's place among the digit's keys), and the row total.
__global__ __launch_bounds__(kRsThreads) void k_rs_rowscan(int32_t* __restrict__ hist, int32_t ntile,
                                                           int32_t* __restrict__ total) {
  __shared__ int32_t buf[kRsThreads];
  const int t = threadIdx.x;
  int32_t* row = hist + (int64_t)blockIdx.x * ntile;
  int32_t carry = 0;
  for (int64_t c0 = 0; c0 < ntile; c0 += kRsThreads) {
    const int64_t k = c0 + t;
    const int32_t v = k < ntile ? row[k] : 0;
    buf[t] = v;
    __syncthreads();
    for (int o = 1; o < kRsThreads; o <<= 1) {
      const int32_t u = t >= o ? buf[t - o] : 0;
      __syncthreads();
      buf[t] += u;
      __syncthreads();
    }
    if (k < ntile) row[k] = carry + buf[t] - v;
    carry += buf[kRsThreads - 1];
    __syncthreads();
  }
  if (t == 0) total[blockIdx.x] = carry;
}

__global__ __launch_bounds__(kRsThreads) void k_rs_scatter(const uint64_t* __restrict__ kin,
                                                           const int32_t* __restrict__ vin,
                                                           uint64_t* __restrict__ kout, int32_t* __restrict__ vout,
                                                           int32_t n, int shift, const int32_t* __restrict__ offs,
                                                           const int32_t* __restrict__ total, int32_t ntile) {
  __shared__ int32_t first[kRsBuckets];          // the tile's first output slot of each digit
  __shared__ int32_t wcnt[kRsThreads / 64][kRsBuckets];
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  // where each digit starts: the exclusive prefix of the digit totals
  const int32_t tot = total[t];
  first[t] = tot;
  __syncthreads();
  for (int o = 1; o < kRsBuckets; o <<= 1) {
    const int32_t u = t >= o ? first[t - o] : 0;
    __syncthreads();
    first[t] += u;
    __syncthreads();
  }
  const int32_t start = first[t] - tot;
  __syncthreads();
  first[t] = start + offs[(int64_t)t * ntile + blockIdx.x];
  for (int q = 0; q < kRsThreads / 64; ++q) wcnt[q][t] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRsTile + (int64_t)w * 64 * kRsRounds;
  const uint64_t below = (1ull << lane) - 1ull;
  uint64_t key[kRsRounds];
  int32_t val[kRsRounds], rank[kRsRounds];
  int dig[kRsRounds];
#pragma unroll
  for (int r = 0; r < kRsRounds; ++r) {
    const int64_t i = base + r * 64 + lane;
    const bool valid = i < n;
    key[r] = valid ? kin[i] : 0ull;
    val[r] = valid ? vin[i] : 0;
    const int d = (int)((key[r] >> shift) & (kRsBuckets - 1));
    dig[r] = d;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < kRsBits; ++b) {
      const bool bit = (d >> b) & 1;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const int before = __popcll(peers & below);
    const int run = valid ? wcnt[w][d] : 0;
    rank[r] = run + before;
    if (valid && before == 0) wcnt[w][d] = run + __popcll(peers);  // the group's first lane
  }
  __syncthreads();
  // per digit, where each wavefront's keys start within the tile
  int32_t acc = 0;
  for (int q = 0; q < kRsThreads / 64; ++q) {
    const int32_t c = wcnt[q][t];
    wcnt[q][t] = acc;
    acc += c;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRsRounds; ++r) {
    const int64_t i = base + r * 64 + lane;
    if (i < n) {
      const int32_t dst = first[dig[r]] + wcnt[w][dig[r]] + rank[r];
      kout[dst] = key[r];
      vout[dst] = val[r];
    }
  }
}

// ------------------------------------------------------- host helpers -----
struct Alloc {
  TreeScratch& s;
  hipStream_t st;
  bool capturing;
  hipError_t err = hipSuccess;
  template <class T>
  T* get(int slot, int64_t count) {
    if (err != hipSuccess) return nullptr;
    const size_t bytes = (size_t)(count > 0 ? count : 1) * sizeof(T);
    if ((int)s.slots.size() <= slot) {
      if (capturing) {
        err = hipErrorStreamCaptureUnsupported;
        return nullptr;
      }
      s.slots.resize(slot + 1, {nullptr, 0});
    }
    auto& sl = s.slots[slot];
    if (sl.second < bytes) {
      if (capturing) {  // no allocation inside a capture: a call outside it sizes the buffers
        err = hipErrorStreamCaptureUnsupported;
        return nullptr;
      }
      if (sl.first) {
        (void)hipStreamSynchronize(st);
        (void)hipFree(sl.first);
        sl.first = nullptr;
        sl.second = 0;
      }
      const size_t cap = bytes + bytes / 4;
      err = hipMalloc(&sl.first, cap);
      if (err != hipSuccess) return nullptr;
      sl.second = cap;
    }
    return static_cast<T*>(sl.first);
  }
};

enum Slot {
  S_BOXPART, S_BOX, S_KEYS, S_KEYS2, S_IDX, S_IDX2, S_POS, S_MASS, S_IJK, S_CELLS, S_CNT, S_OFF, S_TMP,
  S_GB, S_GE, S_GN, S_GBOX, S_STACK, S_CTR, S_ENDS, S_LVL, S_HIST
};

hipError_t exclusive_sum(hipStream_t st, const int32_t* in, int32_t* out, int64_t n) {
  hipLaunchKernelGGL(k_exscan, dim3(1), dim3(kScanThreads), 0, st, in, out, n, nullptr, 0);
  return hipGetLastError();
}

// Sort (keys, idx) by the low `bits` bits of the keys; returns the buffers
// holding the result (the inputs or the alternates, which are overwritten).
hipError_t radix_sort(Alloc& al, uint64_t* keys, int32_t* idx, uint64_t* keys2, int32_t* idx2, int32_t n, int bits,
                      uint64_t** keys_out, int32_t** idx_out) {
  const int32_t ntile = (n + kRsTile - 1) / kRsTile;
  int32_t* hist = al.get<int32_t>(S_HIST, (int64_t)kRsBuckets * ntile + kRsBuckets);
  if (!hist) return al.err != hipSuccess ? al.err : hipErrorOutOfMemory;
  int32_t* total = hist + (int64_t)kRsBuckets * ntile;
  uint64_t *ka = keys, *kb = keys2;
  int32_t *va = idx, *vb = idx2;
  for (int shift = 0; shift < bits; shift += kRsBits) {
    hipLaunchKernelGGL(k_rs_hist, dim3(ntile), dim3(kRsThreads), 0, al.st, ka, n, shift, hist, ntile);
    hipLaunchKernelGGL(k_rs_rowscan, dim3(kRsBuckets), dim3(kRsThreads), 0, al.st, hist, ntile, total);
    hipLaunchKernelGGL(k_rs_scatter, dim3(ntile), dim3(kRsThreads), 0, al.st, ka, va, kb, vb, n, shift, hist, total,
                       ntile);
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  *keys_out = ka;
  *idx_out = va;
  return hipGetLastError();
}

// the entries at `pos`... of a device array, read to the host (synchronises)
template <class T>
hipError_t read_entries(TreeScratch& s, hipStream_t st, const T* a, int64_t count, T* out) {
  T* h = static_cast<T*>(s.host);
  hipError_t e = hipMemcpyAsync(h, a, count * sizeof(T), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e == hipSuccess)
    for (int64_t k = 0; k < count; ++k) out[k] = h[k];
  return e;
}

}  // namespace

#define NB_TRY(x)                 \
  do {                            \
    hipError_t e_ = (x);          \
    if (e_ != hipSuccess) {       \
      *msg = #x;                  \
      return e_;                  \
    }                             \
  } while (0)

namespace {

// box, keys, the sort along the curve; sorted keys and rows go to *keys_s, *idx_s
hipError_t keys_and_order(Alloc& al, const double* pos, int32_t n, Box** box_out, uint64_t** keys_s,
                          int32_t** idx_s, const char** msg) {
  auto need = [&](void* p) -> hipError_t { return p ? hipSuccess : (al.err != hipSuccess ? al.err : hipErrorOutOfMemory); };
  const int nbb = blocks_for(n, 1024);
  double* part = al.get<double>(S_BOXPART, 6 * nbb);
  Box* box = al.get<Box>(S_BOX, 1);
  uint64_t* keys = al.get<uint64_t>(S_KEYS, n);
  uint64_t* keys2 = al.get<uint64_t>(S_KEYS2, n);
  int32_t* idx = al.get<int32_t>(S_IDX, n);
  int32_t* idx2 = al.get<int32_t>(S_IDX2, n);
  NB_TRY(need(idx2));
  hipLaunchKernelGGL(k_bbox_partial, dim3(nbb), dim3(kTB), 0, al.st, pos, (int64_t)n, part);
  hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(kTB), 0, al.st, part, nbb, box);
  hipLaunchKernelGGL(k_keys, dim3(blocks_for(n)), dim3(kTB), 0, al.st, pos, (int64_t)n, box, keys, idx);
  NB_TRY(hipGetLastError());
  NB_TRY(radix_sort(al, keys, idx, keys2, idx2, n, 3 * kBits, keys_s, idx_s));
  *box_out = box;
  return hipSuccess;
}

}  // namespace

hipError_t tree_sorted_keys(TreeScratch& s, hipStream_t st, const double* pos, int32_t n, uint64_t* keys_out,
                            int32_t* idx_out, const char** msg) {
  *msg = "";
  Alloc al{s, st, false};
  Box* box = nullptr;
  uint64_t* keys_s = nullptr;
  int32_t* idx_s = nullptr;
  hipError_t e = keys_and_order(al, pos, n, &box, &keys_s, &idx_s, msg);
  if (e != hipSuccess) return e;
  NB_TRY(hipMemcpyAsync(keys_out, keys_s, (size_t)n * sizeof(uint64_t), hipMemcpyDeviceToDevice, st));
  NB_TRY(hipMemcpyAsync(idx_out, idx_s, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
  return hipSuccess;
}

hipError_t tree_forces_run(TreeScratch& s, hipStream_t st, const double* pos, const double* mass, int32_t n,
                           double eps2, double theta, int n_crit, double g_frac, bool mixed, double* acc,
                           double* pot, TreeStats* stats, bool capturing, unsigned int* err, const char** msg) {
  *msg = "";
  if (!capturing && !s.host) NB_TRY(hipHostMalloc(&s.host, 64 * sizeof(int64_t), hipHostMallocDefault));
  Alloc al{s, st, capturing};
  auto need = [&](void* p) -> hipError_t { return p ? hipSuccess : (al.err != hipSuccess ? al.err : hipErrorOutOfMemory); };

  // box, keys, sort along the curve
  Box* box = nullptr;
  uint64_t* keys_s = nullptr;
  int32_t* idx_s = nullptr;
  {
    hipError_t e = keys_and_order(al, pos, n, &box, &keys_s, &idx_s, msg);
    if (e != hipSuccess) return e;
  }
  double* pos_s = al.get<double>(S_POS, 3 * (int64_t)n);
  double* mass_s = al.get<double>(S_MASS, n);
  int32_t* ijk_s = al.get<int32_t>(S_IJK, 3 * (int64_t)n);
  NB_TRY(need(ijk_s));
  hipLaunchKernelGGL(k_gather, dim3(blocks_for(n)), dim3(kTB), 0, st, pos, mass, idx_s, (int64_t)n, box, pos_s,
                     mass_s, ijk_s);
  NB_TRY(hipGetLastError());

  // cells, level by level, sized once by a bound: a cell that splits holds
  // more than n_crit particles and the cells of one level are disjoint, so
  // each level has at most n / (n_crit + 1) of them; the leaves hold at least
  // one particle each, so there are at most n.  A level has at most
  // min(n, 8 x that) cells.
  const int64_t inner = n / ((int64_t)n_crit + 1);
  const int64_t cap_cells = 1 + (int64_t)kLevels * inner + n;
  const int64_t per_level = std::min<int64_t>(n, 8 * inner + 8);
  TreeCell* cells = al.get<TreeCell>(S_CELLS, cap_cells);
  int32_t* lvl = al.get<int32_t>(S_LVL, kLevels + 1);
  const int32_t nchunk = (n + kGS - 1) / kGS;
  int32_t* cnt = al.get<int32_t>(S_CNT, std::max<int64_t>(per_level + 1, nchunk));
  int32_t* off = al.get<int32_t>(S_OFF, std::max<int64_t>(per_level + 1, nchunk));
  int32_t* ends = al.get<int32_t>(S_ENDS, 8 * per_level);
  NB_TRY(need(ends));
  hipLaunchKernelGGL(k_root, dim3(1), dim3(64), 0, st, cells, n, ijk_s, box, lvl);
  // grid-stride level kernels: a few hundred blocks cover the largest level
  // and keep the launches of the empty levels below the tree cheap
  const int gcount = blocks_for(8 * per_level, 256), gcell = blocks_for(per_level, 256);
  for (int l = 0; l < kBits; ++l) {
    hipLaunchKernelGGL(k_count_children, dim3(gcount), dim3(kTB), 0, st, cells, lvl, l, keys_s, n_crit, cnt, ends);
    hipLaunchKernelGGL(k_exscan, dim3(1), dim3(kScanThreads), 0, st, cnt, off, (int64_t)0, lvl, l);
    hipLaunchKernelGGL(k_write_children, dim3(gcell), dim3(kTB), 0, st, cells, lvl, l, ends, ijk_s, box, n_crit, off);
  }
  NB_TRY(hipGetLastError());
  // moments from the deepest level up (empty levels return at once)
  for (int l = kBits; l >= 0; --l)
    hipLaunchKernelGGL(k_moments, dim3(gcell), dim3(kTB), 0, st, cells, lvl, l, pos_s, mass_s);
  NB_TRY(hipGetLastError());

  // groups: chunks of 64, halved while wider than g_max (one pass to count,
  // one to write)
  int32_t* gb = al.get<int32_t>(S_GB, n);
  int32_t* ge = al.get<int32_t>(S_GE, n);
  int32_t* gn = al.get<int32_t>(S_GN, 1);
  double* gbox = al.get<double>(S_GBOX, 6 * (int64_t)n);
  NB_TRY(need(gbox));
  const int gblocks = blocks_for((int64_t)nchunk * kGS);
  hipLaunchKernelGGL(k_groups<false>, dim3(gblocks), dim3(kTB), 0, st, n, nchunk, pos_s, box, g_frac, cnt,
                     nullptr, nullptr, nullptr, nullptr);
  NB_TRY(exclusive_sum(st, cnt, off, nchunk));
  hipLaunchKernelGGL(k_groups<true>, dim3(gblocks), dim3(kTB), 0, st, n, nchunk, pos_s, box, g_frac, cnt, off,
                     gb, ge, gn);
  hipLaunchKernelGGL(k_group_box, dim3(blocks_for(n, 1024)), dim3(kTB), 0, st, gb, ge, gn, pos_s, gbox);
  NB_TRY(hipGetLastError());

  // walk and forces: one wavefront per group, groups handed out by a counter
  int dev = 0, num_cus = 0, per_cu = 0;
  NB_TRY(hipGetDevice(&dev));
  NB_TRY(hipDeviceGetAttribute(&num_cus, hipDeviceAttributeMultiprocessorCount, dev));
  if (mixed)
    NB_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_tree_walk_forces<true>, kGS, 0));
  else
    NB_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_tree_walk_forces<false>, kGS, 0));
  int64_t grid = (int64_t)(num_cus > 0 ? num_cus : 1) * (per_cu > 0 ? per_cu : 1);
  // the counter hands out every group whatever the grid; a chunk of 64 rarely
  // splits into more than two groups, so more workgroups would mostly find none
  if (grid > 2 * (int64_t)nchunk) grid = 2 * (int64_t)nchunk;
  const int32_t cap = (int32_t)(cap_cells < kStackCap ? cap_cells : kStackCap);
  int32_t* stack = al.get<int32_t>(S_STACK, grid * cap);
  unsigned long long* ctr = al.get<unsigned long long>(S_CTR, 4);
  NB_TRY(need(ctr));
  NB_TRY(need(stack));
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, ctr, 4);
  if (mixed)
    hipLaunchKernelGGL(k_tree_walk_forces<true>, dim3((unsigned)grid), dim3(kGS), 0, st, gb, ge, gn, gbox,
                       cells, theta, pos_s, mass_s, eps2, idx_s, stack, cap, ctr, err, acc, pot);
  else
    hipLaunchKernelGGL(k_tree_walk_forces<false>, dim3((unsigned)grid), dim3(kGS), 0, st, gb, ge, gn, gbox,
                       cells, theta, pos_s, mass_s, eps2, idx_s, stack, cap, ctr, err, acc, pot);
  NB_TRY(hipGetLastError());
  if (!stats) return hipSuccess;
  // counts for the caller (synchronises)
  unsigned long long c[3];
  NB_TRY(read_entries(s, st, ctr + 1, 3, c));
  if (c[2]) {
    *msg = "tree walk stack exceeded its bound";
    return hipErrorInvalidValue;
  }
  int32_t lv[kLevels + 1], ng = 0;
  NB_TRY(read_entries(s, st, lvl, kLevels + 1, lv));
  NB_TRY(read_entries(s, st, gn, 1, &ng));
  int depth = 0;
  for (int l = 0; l < kLevels; ++l)
    if (lv[l + 1] > lv[l]) depth = l;
  stats->cells = lv[kLevels];
  stats->groups = ng;
  stats->accepted = (int64_t)c[0];
  stats->opened_leaves = (int64_t)c[1];
  stats->depth = depth;
  return hipSuccess;
}

void tree_scratch_free(TreeScratch& s) {
  for (auto& sl : s.slots)
    if (sl.first) (void)hipFree(sl.first);
  s.slots.clear();
  if (s.host) (void)hipHostFree(s.host);
  s.host = nullptr;
}

}  // namespace nb
