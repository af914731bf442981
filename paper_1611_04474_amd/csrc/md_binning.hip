// Cell binning: a counting sort of the atoms into cells of edge >= r_cut
// (Section 2.1, Fig. 2), stored as flat arrays instead of linked lists (the second
// code transformation of Section 2.2). Positions become a sorted structure of
// arrays (first transformation of Section 2.2): float4/double4 (x, y, z, q), the
// type and the permutation back to the caller's order.
//
// Kernels, in launch order. When the grid fits in an LDS histogram (up to 32,768 cells):
//   k_bin_hist       each block takes a contiguous range of atoms, wraps each coordinate
//                    into [0, L] (one add/subtract of L in the input precision), checks it,
//                    computes the cell and counts it in an LDS histogram (the LDS atomic's
//                    return value is the atom's slot among the block's atoms of that cell);
//                    the histogram and the block's status bits go to the workspace, so no
//                    global atomics are needed;
// then, for grids of at most 1024 cells, the same block also scans its histogram into the
//                    block's start of each cell and writes its atoms in cell order within
//                    its own range of the arrays (so binning is two kernels: this one and
//                    k_cell_sort, which gathers each cell's atoms from the blocks' ranges);
// and for larger grids
//   k_bin_colscan    per cell, the blocks' exclusive offsets and the total (64 cells per
//                    workgroup);
//   k_bin_scan       one workgroup: exclusive scan of the totals -> cell_start, the launch
//                    order, the LJ table and the status word;
//   k_scatter        each atom to its cell's range.
// Beyond 32,768 cells, k_setup (clears the counters) and k_bin_count (one global atomic per
// atom) take the place of k_bin_hist, and k_bin_scan and k_scatter follow. Last:
//   k_cell_sort      one workgroup per cell: orders the cell's atoms by (z half of the cell,
//                    wrapped x, original index) -- a total order, so every later sum runs
//                    in a reproducible order, and each half of a row of cells along x is
//                    sorted in x, which lets the pair kernel bound the candidates of a group
//                    of home atoms by an x-window per half-row -- writes the sorted arrays
//                    and the number of atoms in the lower z half. On grids of at most 1024
//                    cells its workgroups first gather the cell's atoms (their start is the
//                    sum of the blocks' starts of the cell), and one more workgroup, the
//                    first, writes the launch order, the mixed Lennard-Jones table
//                    (Lorentz-Berthelot) and the status word.
// Within a cell's range the atoms come in arbitrary order (the LDS atomics' order) until the
// in-cell sort; the launch order puts the cells longest first (atom counts, or the last pair
// kernel's measured times on small grids), so that the last workgroups to run are short ones.
#include "md_common.hpp"

namespace md {
namespace {

template <typename Real>
__device__ inline Real wrap_coord(Real x, Real L, uint32_t& st) {
  if (x != x) {
    st |= MD_STATUS_NAN;
    return Real(0);
  }
  if (x < -L || x >= Real(2) * L) {
    st |= MD_STATUS_OUT_OF_BOX;
    return Real(0);
  }
  if (x < Real(0)) return x + L;   // one rounding in the input precision
  if (x >= L) return x - L;        // exact
  return x + Real(0);              // -0 becomes +0
}

template <typename Real>
__device__ inline int cell_coord(Real x, Real inv_w, int n) {
  int c = (int)(x * inv_w);
  c = c < 0 ? 0 : c;
  return c > n - 1 ? n - 1 : c;
}

// Cell of an atom from its raw coordinates and type (which are checked).
template <typename Real>
__device__ inline int cell_from(const SysArgs<Real>& a, Real x0, Real y0, Real z0, int t,
                                uint32_t& st) {
  const Real x = wrap_coord(x0, a.L[0], st);
  const Real y = wrap_coord(y0, a.L[1], st);
  const Real z = wrap_coord(z0, a.L[2], st);
  if (t < 0 || t >= a.n_types) st |= MD_STATUS_BAD_TYPE;
  const int cx = cell_coord(x, a.inv_w[0], a.nx);
  const int cy = cell_coord(y, a.inv_w[1], a.ny);
  const int cz = cell_coord(z, a.inv_w[2], a.nz);
  return (cz * a.ny + cy) * a.nx + cx;
}

template <typename Real>
__device__ inline int cell_of(const SysArgs<Real>& a, int64_t i, uint32_t& st) {
  return cell_from(a, a.pos_in[3 * i + 0], a.pos_in[3 * i + 1], a.pos_in[3 * i + 2],
                   a.type_in[i], st);
}

// Exclusive prefix sum of one value per thread over a workgroup of kWaves waves: a scan
// within each wave, then the wave totals through LDS (s_tot holds kWaves values). *total
// gets the sum of all.
template <int kWaves>
__device__ inline int32_t block_scan_excl_w(int32_t v, int32_t* s_tot, int32_t* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int32_t y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) s_tot[w] = x;
  __syncthreads();
  int32_t before = 0, all = 0;
#pragma unroll
  for (int k = 0; k < kWaves; ++k) {
    const int32_t tk = s_tot[k];
    before += k < w ? tk : 0;
    all += tk;
  }
  __syncthreads();   // s_tot may be reused after this
  *total = all;
  return before + x - v;
}

// The same over a 1024-thread workgroup.
__device__ inline int32_t block_scan_excl(int32_t v, int32_t* s_tot, int32_t* total) {
  return block_scan_excl_w<16>(v, s_tot, total);
}

// Grids of at most kScanFused cells binned with per-block histograms skip the scan
// kernels: each histogram block scans its own counts and writes its atoms in cell order
// within its range, and the in-cell sort gathers every cell from the blocks' ranges.
// Larger grids go through k_bin_colscan, k_bin_scan and k_scatter.
constexpr int kScanFused = 1024;

template <typename Real>
__host__ __device__ inline bool scan_fused(const SysArgs<Real>& a) {
  return a.bin_blocks > 0 && a.n_cells <= kScanFused;
}

// z half of an atom in its cell: 1 if 2 z n_z / L_z reaches the cell's middle.
template <typename Real>
__device__ inline int z_half(const SysArgs<Real>& a, Real z, int cz) {
  return (int)(z * a.inv_w[2] * Real(2)) >= 2 * cz + 1 ? 1 : 0;
}

// Sort key of atom i of cell cz (z index) with wrapped x and z: (z half, x as float32
// bits, original index) in bits 63, 62..31 and 30..0. Wrapped x is >= +0, where the bits
// of a float order as its value (31 bits: the sign bit is 0).
template <typename Real>
__device__ inline unsigned long long sort_key(const SysArgs<Real>& a, int32_t i, float x, Real z,
                                              int cz) {
  return ((unsigned long long)z_half(a, z, cz) << 63) |
         ((unsigned long long)__builtin_bit_cast(uint32_t, x + 0.f) << 31) | (uint32_t)i;
}

// A four-component record with streaming stores (written once, read by the next kernels).
template <typename Real>
__device__ inline void store_nt(P4<Real>* dst, const P4<Real>& v) {
  __builtin_nontemporal_store(v.x, &dst->x);
  __builtin_nontemporal_store(v.y, &dst->y);
  __builtin_nontemporal_store(v.z, &dst->z);
  __builtin_nontemporal_store(v.w, &dst->w);
}

// Atom i (of cell c) goes to slot `slot` of the cell-major arrays that precede the in-cell
// sort: its sort key and type as one 16-byte record, and its wrapped (x, y, z, q).
// kNt: streaming stores (grids of at most kScanFused cells, where each block writes its own
// range and they measured faster); larger grids' k_scatter needs L2 to merge the partial
// lines of its scattered stores. A compile-time choice: a run-time branch between the two
// store forms lets the compiler merge them and drop the hint.
template <bool kNt, typename Real>
__device__ inline void put_atom(const SysArgs<Real>& a, int64_t i, int c, int32_t slot, Real x,
                                Real y, Real z, Real q, int t) {
  const int cz = c / (a.nx * a.ny);   // fewer than 2^24 cells
  uint32_t st = 0;
  P4<Real> p;
  p.x = wrap_coord(x, a.L[0], st);
  p.y = wrap_coord(y, a.L[1], st);
  p.z = wrap_coord(z, a.L[2], st);
  p.w = q;
  if (t < 0 || t >= a.n_types) t = 0;
  const UKey uk{sort_key(a, (int32_t)i, (float)p.x, p.z, cz), t, 0};
  if constexpr (kNt) {
    __builtin_nontemporal_store(uk.key, &a.ukey[slot].key);
    __builtin_nontemporal_store(uk.type, &a.ukey[slot].type);
    store_nt(&a.upos[slot], p);
  } else {
    a.ukey[slot] = uk;
    a.upos[slot] = p;
  }
}

// Clears the per-atom accumulators that the pair kernels add into.
template <typename Real>
__device__ inline void clear_atom(const SysArgs<Real>& a, int64_t i) {
  if (a.flags & MD_ACCUM_F32_ATOMIC) {
    a.facc[i] = 0.f;
    a.facc[a.n + i] = 0.f;
    a.facc[2 * a.n + i] = 0.f;
  }
  if (a.half_shell) {
    // three sums, of one 64-bit word each in float32 and two in float64
    for (int c = 0; c < (sizeof(Real) == 8 ? 6 : 3); ++c) a.acc64[c * a.n + i] = 0;
  }
  if (a.flags & MD_DIAG_COUNTERS) a.paircount[a.n + i] = 0;
}

// kBinThreads threads per block; a block's atoms are taken kHistPer per thread at a time,
// all their loads issued before any of them is binned (the chunk is a multiple of
// kBinThreads kHistPer atoms).
constexpr int kHistPer = kBinChunkUnit / kBinThreads;

// Grids of at most kScanFused cells (scan_fused): after counting, the block scans its
// counts into its start of each cell, bhist[blk][0 .. n_cells] (row n_cells + 1 long, the
// last entry the block's atom count), and writes each of its atoms with its sort key to
// position blk bin_chunk + (block's start of its cell) + (its slot in the cell) of the
// unsorted arrays. A block of one round keeps its atoms in registers meanwhile; longer
// blocks store each atom's cell and slot and read them back. The per-atom sums are cleared
// by the in-cell sort then. Larger grids: the histogram goes to bhist[blk][0 .. n_cells - 1]
// and the cell and slot of each atom to cell[] and rank[], and the block clears its atoms'
// per-atom sums.
template <typename Real>
__device__ inline void bin_hist(const SysArgs<Real>& a, int64_t blk) {
  extern __shared__ int32_t s_h[];   // [n_cells] counts, then the status bits
  __shared__ int32_t s_tot[kBinThreads / 64];
  const int nc = (int)a.n_cells;
  const int tid = threadIdx.x;
  const bool local = scan_fused(a);
  const bool regs = local && a.bin_chunk == (int64_t)kBinThreads * kHistPer;
  for (int c = tid; c <= nc; c += kBinThreads) s_h[c] = 0;
  __syncthreads();
  const int64_t i0 = blk * a.bin_chunk;
  const int64_t i1 = i0 + a.bin_chunk < a.n ? i0 + a.bin_chunk : a.n;
  uint32_t st = 0;
  Real x[kHistPer], y[kHistPer], z[kHistPer], q[kHistPer];
  int ty[kHistPer], c[kHistPer], rk[kHistPer];
  for (int64_t r0 = i0; r0 < i1; r0 += kBinThreads * kHistPer) {
#pragma unroll
    for (int u = 0; u < kHistPer; ++u) {
      // past the end: a repeat of the block's last atom, whose cell and status bits are
      // already its own (nothing is stored for it)
      int64_t i = r0 + u * kBinThreads + tid;
      i = i < i1 ? i : i1 - 1;
      x[u] = a.pos_in[3 * i + 0];
      y[u] = a.pos_in[3 * i + 1];
      z[u] = a.pos_in[3 * i + 2];
      ty[u] = a.type_in[i];
      if (regs) q[u] = a.q_in[i];
    }
#pragma unroll
    for (int u = 0; u < kHistPer; ++u) c[u] = cell_from(a, x[u], y[u], z[u], ty[u], st);
#pragma unroll
    for (int u = 0; u < kHistPer; ++u) {
      const int64_t i = r0 + u * kBinThreads + tid;
      if (i < i1) {
        rk[u] = atomicAdd(&s_h[c[u]], 1);
        if (!regs) {
          a.cell[i] = c[u];
          a.rank[i] = rk[u];
        }
        if (!local) clear_atom(a, i);
      }
    }
  }
  if (st) atomicOr(reinterpret_cast<uint32_t*>(&s_h[nc]), st);
  __syncthreads();
  if (!local) {
    int32_t* hb = a.bhist + blk * nc;
    for (int cc = tid; cc < nc; cc += kBinThreads) hb[cc] = s_h[cc];
    if (tid == 0) a.bstat[blk] = (uint32_t)s_h[nc];
    return;
  }
  // the block's start of each cell: kCellsPer consecutive cells per thread (nc <= 1024)
  constexpr int kCellsPer = kScanFused / kBinThreads;
  static_assert(kCellsPer * kBinThreads == kScanFused, "cells per thread");
  const uint32_t stb = (uint32_t)s_h[nc];
  const int c0 = kCellsPer * tid;
  int32_t v[kCellsPer], sum = 0;
#pragma unroll
  for (int k = 0; k < kCellsPer; ++k) {
    v[k] = c0 + k < nc ? s_h[c0 + k] : 0;
    sum += v[k];
  }
  int32_t all;
  int32_t ex = block_scan_excl_w<kBinThreads / 64>(sum, s_tot, &all);
  int32_t* lrow = a.bhist + blk * (int64_t)(nc + 1);
#pragma unroll
  for (int k = 0; k < kCellsPer; ++k) {
    if (c0 + k < nc) {
      s_h[c0 + k] = ex;
      lrow[c0 + k] = ex;
    }
    ex += v[k];
  }
  if (tid == 0) {
    lrow[nc] = all;
    a.bstat[blk] = stb;
  }
  __syncthreads();
  if (regs) {
#pragma unroll
    for (int u = 0; u < kHistPer; ++u) {
      const int64_t i = i0 + u * kBinThreads + tid;
      if (i < i1) put_atom<true>(a, i, c[u], (int32_t)(i0 + s_h[c[u]] + rk[u]), x[u], y[u], z[u], q[u], ty[u]);
    }
    return;
  }
  for (int64_t i = i0 + tid; i < i1; i += kBinThreads) {
    const int ci = a.cell[i];
    put_atom<true>(a, i, ci, (int32_t)(i0 + s_h[ci] + a.rank[i]), a.pos_in[3 * i + 0],
             a.pos_in[3 * i + 1], a.pos_in[3 * i + 2], a.q_in[i], a.type_in[i]);
  }
}

template <typename Real>
__global__ __launch_bounds__(kBinThreads) void k_bin_hist(SysArgs<Real> a) {
  bin_hist(a, blockIdx.x);
}

__global__ __launch_bounds__(kBinThreads) void k_bin_hist_batch(Batch<float> b) {
  int64_t blk;
  const int s = b.pick(blockIdx.x, blk);
  bin_hist(b.sys[s], blk);
}

template <typename Real>
__global__ void k_setup(SysArgs<Real> a) {
  int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t c = tid; c < a.n_cells; c += stride) a.count[c] = 0;
  for (int64_t i = tid; i < a.n; i += stride) clear_atom(a, i);
  if (tid == 0) {
    a.hdr->status = 0;
    for (int k = 0; k < 5; ++k) a.hdr->diag[k] = 0;
    a.hdr->clock[0] = a.hdr->clock[1] = 0;
  }
}

template <typename Real>
__global__ void k_bin_count(SysArgs<Real> a) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  uint32_t st = 0;
  const int c = cell_of(a, i, st);
  a.cell[i] = c;
  a.rank[i] = atomicAdd(&a.count[c], 1);
  if (st) atomicOr(&a.hdr->status, st);
}

// Workgroups of k_bin_colscan for one system (0 when the scatter does the scan).
template <typename Real>
__host__ __device__ inline int64_t colscan_blocks(const SysArgs<Real>& a) {
  return a.bin_blocks > 0 && !scan_fused(a) ? (a.n_cells + 63) / 64 : 0;
}

// Per-block histograms of large grids: workgroup blk (1024 threads) takes cells
// 64 blk .. 64 blk + 63, one per lane. Wave w sums its share of the blocks' counts of the
// lane's cell (up to 64 blocks, all loads in flight), the 16 wave sums are scanned through
// LDS, and the counts become each block's exclusive offset within the cell (in place);
// their total is the cell count.
template <typename Real>
__device__ inline void bin_colscan(const SysArgs<Real>& a, int64_t blk) {
  static_assert(kBinMaxBlocks <= 16 * 64, "a wave sums at most 64 blocks");
  __shared__ int32_t s_col[16][64];
  const int t = threadIdx.x, lane = t & 63;
  const int w = __builtin_amdgcn_readfirstlane(t >> 6);   // uniform: row addresses in SGPRs
  const int64_t nc = a.n_cells;
  const int B = a.bin_blocks;
  const int64_t c = blk * 64 + lane;
  const bool cv = c < nc;
  const int per = (B + 15) / 16;   // blocks per wave
  const int b0 = w * per;
  int32_t v[64];
  int32_t sum = 0;
#pragma unroll
  for (int r = 0; r < 64; ++r) {
    const int b = b0 + r;
    v[r] = (r < per && b < B && cv) ? a.bhist[(int64_t)b * nc + c] : 0;
    sum += v[r];
  }
  s_col[w][lane] = sum;
  __syncthreads();
  int32_t base = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int32_t x = s_col[k][lane];
    base += k < w ? x : 0;
    tot += x;
  }
#pragma unroll
  for (int r = 0; r < 64; ++r) {
    const int b = b0 + r;
    if (r < per && b < B && cv) a.bhist[(int64_t)b * nc + c] = base;
    base += v[r];
  }
  if (w == 0 && cv) a.count[c] = tot;
}

template <typename Real>
__global__ __launch_bounds__(1024) void k_bin_colscan(SysArgs<Real> a) {
  bin_colscan(a, blockIdx.x);
}

__global__ __launch_bounds__(1024) void k_bin_colscan_batch(Batch<float> b) {
  int64_t blk;
  const int s = b.pick(blockIdx.x, blk);
  bin_colscan(b.sys[s], blk);
}

// Whether cost[] holds the pair kernel's times of the last evaluation on this grid (a
// workspace fresh from the caller holds anything: then the key rarely matches, and a false
// match only changes the launch order).
template <typename Real>
__device__ inline bool have_costs(const SysArgs<Real>& a) {
  return a.hdr->cost_key == kCostKey && a.hdr->cost_cells == (uint32_t)a.n_cells;
}

// Launch-order key of a cell from its time in units of the 100 MHz clock: bins of 160 ns,
// so the 1024 bins of the order's counting sort span 164 us per cell (longer ones share
// the first bin).
__device__ inline uint32_t cost_key(uint32_t ticks) { return ticks >> 4; }

// The cells' launch order for the pair kernel, the mixed LJ table and (own_header) the
// status word: the end of the scan, by one workgroup of kThreads threads (s_tot holds
// kThreads / 64 values). key(c) is cell c's expected cost: its atom count, or (grids of at
// most kScanFused cells) its time in the last pair kernel when known; st_lane (threads
// 0 .. 63) carries the histogram blocks' status bits from block_status.
template <int kThreads, typename Real, typename Key>
__device__ inline void scan_tail(const SysArgs<Real>& a, const TypeTable& tt, int own_header,
                                 int32_t* s_tot, int32_t* s_bin, Key key, uint32_t st_lane) {
  const int t = threadIdx.x;
  const int64_t nc = a.n_cells;
  // counting sort of the cells by decreasing key (keys clamped to kOrderBins - 1); the
  // order within a bin is arbitrary, which only changes which compute unit takes a cell,
  // never a result. Longest first lets the short cells fill the tail.
  constexpr int kOrderBins = 1024;
  constexpr int kPerT = kOrderBins / kThreads;   // bins per thread, consecutive (s_bin holds
                                                 // kOrderBins)
#pragma unroll
  for (int k = 0; k < kPerT; ++k) s_bin[kPerT * t + k] = 0;
  __syncthreads();
  auto bin = [&](int64_t c) {
    const uint32_t v = key(c);
    return kOrderBins - 1 - (int)(v < kOrderBins - 1 ? v : kOrderBins - 1);
  };
  for (int64_t c = t; c < nc; c += kThreads) atomicAdd(&s_bin[bin(c)], 1);
  __syncthreads();
  {
    int32_t v[kPerT], sum = 0, all;
#pragma unroll
    for (int k = 0; k < kPerT; ++k) {
      v[k] = s_bin[kPerT * t + k];
      sum += v[k];
    }
    int32_t excl = block_scan_excl_w<kThreads / 64>(sum, s_tot, &all);
#pragma unroll
    for (int k = 0; k < kPerT; ++k) {
      s_bin[kPerT * t + k] = excl;   // each thread rewrites only its own bins, read above
      excl += v[k];
    }
    __syncthreads();
  }
  for (int64_t c = t; c < nc; c += kThreads) {
    const int32_t pos = atomicAdd(&s_bin[bin(c)], 1);
    a.order[pos] = (int32_t)c;
  }
  const int nt = a.n_types;
  for (int e = t; e < nt * nt; e += kThreads) {
    const int ti = e / nt, tj = e % nt;
    const double sg = 0.5 * (tt.sigma[ti] + tt.sigma[tj]);
    const double ep = sqrt(tt.eps[ti] * tt.eps[tj]);
    const double s2 = sg * sg, s6 = s2 * s2 * s2;
    a.lj[2 * e + 0] = (Real)(4.0 * ep * s6 * s6);
    a.lj[2 * e + 1] = (Real)(4.0 * ep * s6);
  }
  if (own_header && t < 64) {
    uint32_t st = st_lane;
    for (int o = 32; o > 0; o >>= 1) st |= __shfl_xor(st, o);
    if (t == 0) a.hdr->status = st;
    if (t < 5) a.hdr->diag[t] = 0;
    if (t < 2) a.hdr->clock[t] = 0;
  }
}

// Status bits of the histogram blocks t, t + 64, ... (threads t < 64 of a workgroup),
// loaded by block_status and combined by Status::bits where they are needed, so that the
// loads overlap others.
struct Status {
  static_assert(kBinMaxBlocks <= 16 * 64, "16 loads per thread");
  uint32_t v[16];
  __device__ uint32_t bits() const {
    uint32_t st = 0u;
#pragma unroll
    for (int k = 0; k < 16; ++k) st |= v[k];
    return st;
  }
};

template <typename Real>
__device__ inline Status block_status(const SysArgs<Real>& a, bool want) {
  Status s;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int b = (int)threadIdx.x + 64 * k;
    s.v[k] = want && threadIdx.x < 64 && b < a.bin_blocks ? a.bstat[b] : 0u;
  }
  return s;
}

// Cell counts of grids of at most kScanLds cells are kept in LDS by the scan kernel.
constexpr int kScanLds = 8192;

// One workgroup of 1024 threads (grids scanned by k_bin_colscan, or binned with global
// atomics): the exclusive scan of the cell counts into start[] (start[n_cells] = n), in
// chunks of 4096 with a running carry, then scan_tail. The counts are read into LDS first
// when the grid has at most kScanLds cells.
template <typename Real>
__device__ inline void bin_scan(const SysArgs<Real>& a, const TypeTable& tt, int own_header) {
  __shared__ int32_t s_tot[16];
  __shared__ int32_t s_cnt[kScanLds];
  const int t = threadIdx.x;
  const int64_t nc = a.n_cells;
  const bool in_lds = nc <= kScanLds;
  const Status st_blocks = block_status(a, own_header != 0);
  if (in_lds) {
    for (int c0 = 0; c0 < nc; c0 += 8 * 1024) {
      int32_t v[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int c = c0 + 1024 * k + t;
        v[k] = c < nc ? a.count[c] : 0;
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int c = c0 + 1024 * k + t;
        if (c < nc) s_cnt[c] = v[k];
      }
    }
  }
  __syncthreads();   // the counts staged above are read by other threads below
  auto count = [&](int64_t c) { return in_lds ? s_cnt[c] : a.count[c]; };
  int32_t carry = 0;
  for (int64_t base = 0; base < nc; base += 4096) {
    int32_t v[4];
    int32_t sum = 0;
    for (int k = 0; k < 4; ++k) {
      const int64_t idx = base + 4 * t + k;
      v[k] = idx < nc ? count(idx) : 0;
      sum += v[k];
    }
    int32_t chunk;
    int32_t run = carry + block_scan_excl(sum, s_tot, &chunk);
    for (int k = 0; k < 4; ++k) {
      const int64_t idx = base + 4 * t + k;
      if (idx < nc) a.start[idx] = run;
      run += v[k];
    }
    carry += chunk;
  }
  if (t == 0) a.start[nc] = carry;
  // launch order by atom count: with more than 1024 cells there are several workgroups
  // per compute unit, and the short cells already fill the tail
  __shared__ int32_t s_bin[1024];
  scan_tail<1024>(a, tt, own_header, s_tot, s_bin, [&](int64_t c) { return (uint32_t)count(c); },
            st_blocks.bits());
}

template <typename Real>
__global__ __launch_bounds__(1024) void k_bin_scan(SysArgs<Real> a, TypeTable tt,
                                                   int own_header) {
  bin_scan(a, tt, own_header);
}

__global__ __launch_bounds__(1024) void k_bin_scan_batch(Batch<float> b, TypeTable tt) {
  int64_t blk;
  const int s = b.pick(blockIdx.x, blk);
  bin_scan(b.sys[s], tt, 1);
}

// Each atom goes to its cell's range (in arbitrary order) with its sort key, its wrapped
// (x, y, z, q) and its type, read here in the caller's order (coalesced), so the in-cell
// sort only touches its own cell's range.
// Workgroups are dealt to the 8 XCDs in turn, each with its own L2. Block bid is renumbered
// so that every XCD takes one contiguous range of the nblk blocks (the first nblk % 8 XCDs
// one block more): a bijection on 0..nblk-1, so only the placement changes. The scatter's
// consecutive blocks share a histogram row (bhist[i / bin_chunk]); numbered this way a row
// is fetched into one L2 instead of into up to eight.
__device__ inline int64_t xcd_contiguous(int64_t bid, int64_t nblk) {
  const int64_t x = bid % 8, k = bid / 8, q = nblk / 8, r = nblk % 8;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + k;
}

template <typename Real>
__device__ inline void scatter(const SysArgs<Real>& a, int64_t blk) {
  const int64_t i = blk * 256 + threadIdx.x;
  if (i >= a.n) return;
  const int c = a.cell[i];
  int32_t slot = a.start[c] + a.rank[i];
  if (a.bin_blocks > 0) slot += a.bhist[(i / a.bin_chunk) * a.n_cells + c];
  put_atom<false>(a, i, c, slot, a.pos_in[3 * i + 0], a.pos_in[3 * i + 1], a.pos_in[3 * i + 2],
           a.q_in[i], a.type_in[i]);
}

template <typename Real>
__global__ __launch_bounds__(256) void k_scatter(SysArgs<Real> a) {
  scatter(a, xcd_contiguous(blockIdx.x, gridDim.x));
}

__global__ __launch_bounds__(256) void k_scatter_batch(Batch<float> b) {
  int64_t blk;
  const int s = b.pick(blockIdx.x, blk);
  scatter(b.sys[s], blk);
}

// One workgroup per cell. Each member's position in the cell is the number of members
// with a smaller key (keys are distinct: they hold the atom index), counted over LDS
// chunks of the cell's keys, so any cell occupancy is handled; the member's data then
// move to that position.
// Adds to *s_low the number of lanes of this wave with `low` set: one LDS atomic per wave
// (called by every lane of the wave).
__device__ inline void count_low(int32_t* s_low, bool low) {
  const unsigned long long b = __builtin_amdgcn_ballot_w64(low);
  if ((threadIdx.x & 63) == 0 && b != 0ull) atomicAdd(s_low, (int32_t)__builtin_popcountll(b));
}

// Centre of cell c (the origin the compacted kernel's prefilter is expanded about).
template <typename Real>
__device__ inline P4<Real> cell_centre(const SysArgs<Real>& a, int64_t c) {
  const int32_t cc = (int32_t)c, nx = a.nx, nxy = a.nx * a.ny;
  const int c0 = cc % nx, c1 = (cc / nx) % a.ny, c2 = cc / nxy;
  P4<Real> o;
  o.x = ((Real)c0 + Real(0.5)) * (a.L[0] / (Real)a.nx);
  o.y = ((Real)c1 + Real(0.5)) * (a.L[1] / (Real)a.ny);
  o.z = ((Real)c2 + Real(0.5)) * (a.L[2] / (Real)a.nz);
  o.w = Real(0);
  return o;
}

// The compacted kernel's constants of the atom at sorted position d as a home atom
// (SysArgs::hpre), with o its cell's centre: a = r - o, so that the kernel's expanded-form
// prefilter |r_j - r_i|^2 = c_j - 2 a.(r_j - o) + |a|^2 becomes
// c_j + (-2 a).r_j < rc^2 + margin - |a|^2 + (-2 a).o; and k q and the atom's row of the
// type-pair table.
template <bool kNt, typename Real>
__device__ inline void write_hpre(const SysArgs<Real>& a, const P4<Real>& o, int32_t d,
                                  const P4<Real>& p, int t) {
  const Real rx = p.x - o.x, ry = p.y - o.y, rz = p.z - o.z;
  const Real ax = Real(-2) * rx, ay = Real(-2) * ry, az = Real(-2) * rz;
  P4<Real> h0, h1;
  h0.x = ax;
  h0.y = ay;
  h0.z = az;
  h0.w = (a.rc2 + Real(kPrefilterMargin)) - fma(rz, rz, fma(ry, ry, rx * rx)) +
         (ax * o.x + ay * o.y + az * o.z);
  h1.x = a.coulomb_k * p.w;
  h1.y = int_to_slot<Real>(t * a.n_types);
  h1.z = Real(0);
  h1.w = Real(0);
  if constexpr (kNt) {
    store_nt(&a.hpre[2 * (int64_t)d], h0);
    store_nt(&a.hpre[2 * (int64_t)d + 1], h1);
  } else {
    a.hpre[2 * (int64_t)d] = h0;
    a.hpre[2 * (int64_t)d + 1] = h1;
  }
}

// Threads of a workgroup of k_cell_sort.
constexpr int kSortThreads = 256;
constexpr int kSortChunk = 1024;                      // members ranked in one LDS chunk
constexpr int kHalfB = kSortThreads / 2;              // rank-count buckets per z half
constexpr int kBucketMax = 8;                         // members a bucket holds

// LDS of a k_cell_sort workgroup, one object for every form of the kernel's code (the
// sort's two store forms and the tail), so that it is allocated once: 18.5 KB leaves room
// for eight workgroups per compute unit.
struct SortLds {
  unsigned long long key[kSortChunk];
  int32_t src[kSortChunk];
  int32_t bcnt[2 * kHalfB], bstart[2 * kHalfB];
  uint16_t blist[2 * kHalfB * kBucketMax];
  int32_t tot[kSortThreads / 64];
  int32_t low, over;
};
__device__ inline SortLds& sort_lds() {
  __shared__ SortLds l;
  return l;
}

// kNt: the outputs with streaming stores (grids of at most kScanFused cells).
template <bool kNt, typename Real>
__device__ inline void cell_sort(const SysArgs<Real>& a, int64_t c) {
  constexpr int kChunk = kSortChunk;
  constexpr int kPer = kChunk / kSortThreads;
  // buckets of the rank count: kHalfB per z half, in x order, at most kBucketMax members each
  SortLds& L = sort_lds();
  unsigned long long* s_key = L.key;
  int32_t* s_src = L.src;
  int32_t* s_tot = L.tot;
  int32_t* s_bcnt = L.bcnt;
  int32_t* s_bstart = L.bstart;
  uint16_t* s_blist = L.blist;
  int32_t& s_low = L.low;
  int32_t& s_over = L.over;
  const bool fused = scan_fused(a);
  const int t = threadIdx.x, lane = t & 63;
  int32_t s0, m;
  // the rank count's bucket counters, cleared before the first barrier
  s_bcnt[t] = 0;
  if (t == 0) s_over = 0;
  if (fused) {
    // block b's atoms of this cell are bhist[b][c + 1] - bhist[b][c] of its range, from
    // position b bin_chunk + bhist[b][c]; the cell starts at the sum over the blocks of
    // bhist[b][c] (the atoms in earlier cells). With at most 256 blocks every wave reads
    // them, lane l taking blocks l, l + 64, l + 128, l + 192, and forms the start, the count
    // and the lanes' offsets with lane sums and scans (the first wave then writes the member
    // list); otherwise thread t takes blocks t, t + 256, ... and block scans.
    constexpr int kBPer = kBinMaxBlocks / kSortThreads;
    const int B = a.bin_blocks;
    const bool one_wave = B <= 64 * kBPer;
    const int bstride = one_wave ? 64 : kSortThreads;
    const int64_t row = a.n_cells + 1;
    int32_t ls[kBPer], cb[kBPer];
    int32_t sl = 0, sc = 0;
    const int bi = one_wave ? lane : t;
#pragma unroll
    for (int k = 0; k < kBPer; ++k) {
      const int b = bi + bstride * k;
      ls[k] = cb[k] = 0;
      if (b < B) {
        const int32_t* r = a.bhist + b * row + c;
        ls[k] = r[0];
        cb[k] = r[1] - ls[k];
      }
      sl += ls[k];
      sc += cb[k];
    }
    int32_t off;
    if (one_wave) {
      int32_t inc = sc;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int32_t y = __shfl_up(inc, o);
        if (lane >= o) inc += y;
        sl += __shfl_xor(sl, o);
      }
      off = inc - sc;
      m = __shfl(inc, 63);   // the cell's atom count
      s0 = sl;               // its start
    } else {
      block_scan_excl_w<kSortThreads / 64>(sl, s_tot, &s0);
      off = block_scan_excl_w<kSortThreads / 64>(sc, s_tot, &m);
    }
    if (t == 0) a.start[c] = s0;
    // the members' positions in the unsorted arrays, in LDS, or for a cell of more than
    // kChunk atoms in rank[s0 .. s0 + m) (read back by this workgroup only)
    if (!one_wave || t < 64) {
#pragma unroll
      for (int k = 0; k < kBPer; ++k) {
        const int32_t p0 = (int32_t)((int64_t)(t + bstride * k) * a.bin_chunk) + ls[k];
        if (m <= kChunk) {
#pragma unroll 1
          for (int32_t r = 0; r < cb[k]; ++r) s_src[off + r] = p0 + r;
        } else {
#pragma unroll 1
          for (int32_t r = 0; r < cb[k]; ++r) a.rank[s0 + off + r] = p0 + r;
        }
        off += cb[k];
      }
    }
    __syncthreads();
  } else {
    s0 = a.start[c];
    m = a.start[c + 1] - s0;
    __syncthreads();   // the bucket counters are cleared before any workgroup thread counts
  }
  // position of member e in the unsorted arrays
  auto src = [&](int32_t e) -> int32_t {
    return !fused ? s0 + e : m <= kChunk ? s_src[e] : a.rank[s0 + e];
  };
  const P4<Real> o = cell_centre(a, c);
  // the cell's x range (its lower face and width), for the rank count's buckets
  const Real cell_w = a.L[0] / (Real)a.nx;
  const Real cell_x0 = o.x - Real(0.5) * cell_w;
  if (t == 0) s_low = 0;
  if (m == 0) {
    if (t == 0) a.zsplit[c] = 0;
    return;
  }
  if (m <= kChunk) {
    // the whole cell in one LDS chunk: each member's key, position and type are loaded
    // once, together, and the keys go to LDS from registers
    const int kk = (m + kSortThreads - 1) / kSortThreads;   // member slots in use (uniform)
    unsigned long long my_key[kPer];
    Real px[kPer], py[kPer], pz[kPer], pq[kPer];
    int32_t my_t[kPer], my_rank[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int32_t e = t + kSortThreads * k;
      const bool in = k < kk && e < m;
      const int32_t sp = src(in ? e : 0);   // m >= 1 here: a valid member
      const UKey u = a.ukey[sp];
      my_key[k] = in ? u.key : ~0ull;
      const P4<Real> p = a.upos[sp];
      px[k] = p.x;
      py[k] = p.y;
      pz[k] = p.z;
      pq[k] = p.w;
      my_t[k] = u.type;
      my_rank[k] = 0;
    }
    // slots m .. kSortThreads kk - 1 (a multiple of 8) hold ~0, which is below no key
#pragma unroll
    for (int k = 0; k < kPer; ++k)
      if (k < kk) s_key[t + kSortThreads * k] = my_key[k];
    // rank = members in earlier buckets + smaller keys in the member's own bucket; the
    // bucket, from the z half and x of the key, never decreases as the key grows
    const float bx0 = (float)cell_x0, bsc = (float)(kHalfB / cell_w);
    int bk[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int32_t e = t + kSortThreads * k;
      bk[k] = 0;
      if (k < kk && e < m) {
        const float x = __uint_as_float((uint32_t)(my_key[k] >> 31) & 0x7fffffffu);
        const int xb = min(max((int)((x - bx0) * bsc), 0), kHalfB - 1);
        bk[k] = (int)(my_key[k] >> 63) * kHalfB + xb;
        const int sl = atomicAdd(&s_bcnt[bk[k]], 1);
        if (sl < kBucketMax)
          s_blist[bk[k] * kBucketMax + sl] = (uint16_t)e;
        else
          s_over = 1;
      }
    }
    __syncthreads();
    if (s_over == 0) {
      // bucket starts: the first wave scans the counts, four consecutive buckets per lane
      static_assert(2 * kHalfB == 4 * 64, "four buckets per lane");
      if (t < 64) {
        int32_t v[4], sum = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          v[k] = s_bcnt[4 * t + k];
          sum += v[k];
        }
        int32_t inc = sum;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
          const int32_t y = __shfl_up(inc, o);
          if (t >= o) inc += y;
        }
        int32_t ex = inc - sum;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          s_bstart[4 * t + k] = ex;
          ex += v[k];
        }
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < kPer; ++k) {
        const int32_t e = t + kSortThreads * k;
        if (k < kk && e < m) {
          const int b = bk[k], nb = s_bcnt[b];
          int r = s_bstart[b];
          for (int j = 0; j < nb; ++j) r += s_key[s_blist[b * kBucketMax + j]] < my_key[k];
          my_rank[k] = r;
        }
      }
    } else {
      // a crowded bucket: every member counts every smaller key of the cell
      for (int32_t e = 0; e < m; e += 8) {
        unsigned long long kx[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) kx[u] = s_key[e + u];
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
          if (k < kk) {
#pragma unroll
            for (int u = 0; u < 8; ++u) my_rank[k] += kx[u] < my_key[k];
          }
        }
      }
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int32_t e = t + kSortThreads * k;
      const bool in = k < kk && e < m;
      count_low(&s_low, in && !(my_key[k] >> 63));
      if (!in) continue;
      const int32_t d = s0 + my_rank[k];
      P4<Real> p;
      p.x = px[k];
      p.y = py[k];
      p.z = pz[k];
      p.w = pq[k];
      if constexpr (kNt) {
        store_nt(&a.pos[d], p);
        __builtin_nontemporal_store(my_t[k], &a.type[d]);
        __builtin_nontemporal_store((int32_t)(my_key[k] & 0x7fffffffull), &a.perm[d]);
      } else {
        a.pos[d] = p;
        a.type[d] = my_t[k];
        a.perm[d] = (int32_t)(my_key[k] & 0x7fffffffull);
      }
      if (a.compact) write_hpre<kNt>(a, o, d, p, my_t[k]);
      if (fused) clear_atom(a, d);
    }
    __syncthreads();
    if (t == 0) a.zsplit[c] = s_low;
    return;
  }
  for (int32_t a0 = 0; a0 < m; a0 += kChunk) {
    const int kk = min(kPer, (m - a0 + kSortThreads - 1) / kSortThreads);   // slots in use
    unsigned long long my_key[kPer];
    int32_t my_rank[kPer];
    for (int k = 0; k < kPer; ++k) {
      const int32_t e = a0 + t + kSortThreads * k;
      my_key[k] = (k < kk && e < m) ? a.ukey[src(e)].key : ~0ull;
      my_rank[k] = 0;
    }
    for (int32_t b0 = 0; b0 < m; b0 += kChunk) {
      const int32_t mb = min(kChunk, m - b0);
      __syncthreads();
      for (int32_t e = t; e < mb; e += kSortThreads) s_key[e] = a.ukey[src(b0 + e)].key;
      for (int32_t e = mb + t; e < ((mb + 3) & ~3); e += kSortThreads) s_key[e] = ~0ull;
      __syncthreads();
      for (int32_t e = 0; e < mb; e += 4) {
        const unsigned long long k0 = s_key[e], k1 = s_key[e + 1], k2 = s_key[e + 2],
                                 k3 = s_key[e + 3];
        for (int k = 0; k < kPer; ++k) {
          if (k < kk)
            my_rank[k] += (k0 < my_key[k]) + (k1 < my_key[k]) + (k2 < my_key[k]) + (k3 < my_key[k]);
        }
      }
    }
    for (int k = 0; k < kPer; ++k) {
      const int32_t e = a0 + t + kSortThreads * k;
      const bool in = k < kk && e < m;
      count_low(&s_low, in && !(my_key[k] >> 63));
      if (!in) continue;
      const int32_t d = s0 + my_rank[k];
      const int32_t sp = src(e);
      const P4<Real> p = a.upos[sp];
      const int32_t ty = a.ukey[sp].type;
      if constexpr (kNt) {
        store_nt(&a.pos[d], p);
        __builtin_nontemporal_store(ty, &a.type[d]);
        __builtin_nontemporal_store((int32_t)(my_key[k] & 0x7fffffffull), &a.perm[d]);
      } else {
        a.pos[d] = p;
        a.type[d] = ty;
        a.perm[d] = (int32_t)(my_key[k] & 0x7fffffffull);
      }
      if (a.compact) write_hpre<kNt>(a, o, d, p, ty);
      if (fused) clear_atom(a, d);
    }
  }
  __syncthreads();
  if (t == 0) a.zsplit[c] = s_low;
}

// The end of the binning on grids of at most kScanFused cells, by the first workgroup of
// k_cell_sort alongside the cells' (which write their own starts): start[n_cells], then
// scan_tail with each cell's order key, its time in the last pair kernel when known, else
// its atom count summed over the histogram blocks.
template <typename Real>
__device__ inline void bin_tail(const SysArgs<Real>& a, const TypeTable& tt) {
  static_assert(sizeof(SortLds::key) >= 4 * kScanFused && sizeof(SortLds::src) >= 4 * 1024,
                "the tail's arrays fit the sort's");
  SortLds& L = sort_lds();
  uint32_t* s_k = reinterpret_cast<uint32_t*>(L.key);   // [kScanFused] order keys
  int32_t* s_tot = L.tot;
  const int t = threadIdx.x;
  const int nc = (int)a.n_cells, B = a.bin_blocks;
  const int64_t row = nc + 1;
  const Status st_blocks = block_status(a, true);
  const bool by_cost = have_costs(a);
  if (t == 0) a.start[nc] = (int32_t)a.n;
  for (int c = t; c < nc; c += kSortThreads) {
    uint32_t key = 0;
    if (by_cost) {
      key = cost_key(a.cost[c]);
    } else {
      for (int b0 = 0; b0 < B; b0 += 32) {
        int32_t v[32];
#pragma unroll
        for (int r = 0; r < 32; ++r) {
          const int32_t* p = a.bhist + (b0 + r) * row + c;
          v[r] = b0 + r < B ? p[1] - p[0] : 0;
        }
#pragma unroll
        for (int r = 0; r < 32; ++r) key += (uint32_t)v[r];
      }
    }
    s_k[c] = key;
  }
  __syncthreads();
  scan_tail<kSortThreads>(a, tt, 1, s_tot, L.src, [&](int64_t c) { return s_k[c]; },
                          st_blocks.bits());
}

// Block blk of k_cell_sort: with the fused scan, block 0 ends the binning and block c + 1
// sorts cell c; otherwise block c sorts cell c.
template <typename Real>
__device__ inline void cell_sort_or_tail(const SysArgs<Real>& a, const TypeTable& tt, int64_t blk) {
  if (!scan_fused(a)) {
    cell_sort<false>(a, blk);
  } else if (blk == 0) {
    bin_tail(a, tt);
  } else {
    cell_sort<true>(a, blk - 1);
  }
}

template <typename Real>
__host__ __device__ inline int64_t sort_blocks(const SysArgs<Real>& a) {
  return a.n_cells + (scan_fused(a) ? 1 : 0);
}

template <typename Real>
__global__ __launch_bounds__(kSortThreads) void k_cell_sort(SysArgs<Real> a, TypeTable tt) {
  cell_sort_or_tail(a, tt, blockIdx.x);
}

__global__ __launch_bounds__(kSortThreads) void k_cell_sort_batch(Batch<float> b, TypeTable tt) {
  int64_t blk;
  const int s = b.pick(blockIdx.x, blk);
  cell_sort_or_tail(b.sys[s], tt, blk);
}

}  // namespace

TypeTable make_type_table(const md_params* p) {
  TypeTable tt;
  for (int t = 0; t < kMaxTypes; ++t) {
    tt.sigma[t] = t < p->n_types ? p->sigma[t] : 0.0;
    tt.eps[t] = t < p->n_types ? p->epsilon[t] : 0.0;
  }
  return tt;
}

template <typename Real>
hipError_t launch_binning(const SysArgs<Real>& a, const TypeTable& tt, hipStream_t stream) {
  int own_header = 1;
  if (a.n > 0 && a.bin_blocks > 0) {
    const size_t shmem = sizeof(int32_t) * (size_t)(a.n_cells + 1);
    hipLaunchKernelGGL(k_bin_hist<Real>, dim3((unsigned)a.bin_blocks), dim3(kBinThreads), shmem, stream,
                       a);
  } else if (a.n > 0) {
    int64_t work = a.n_cells > a.n ? a.n_cells : a.n;
    int64_t blocks = (work + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_setup<Real>, dim3((unsigned)blocks), dim3(256), 0, stream, a);
    hipLaunchKernelGGL(k_bin_count<Real>, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0,
                       stream, a);
    own_header = 0;
  }
  SysArgs<Real> as = a;
  if (a.n == 0) {
    // nothing binned: every cell is empty
    as.bin_blocks = 0;
    int64_t blocks = (a.n_cells + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_setup<Real>, dim3((unsigned)blocks), dim3(256), 0, stream, as);
  }
  if (!scan_fused(as)) {
    if (colscan_blocks(as) > 0)
      hipLaunchKernelGGL(k_bin_colscan<Real>, dim3((unsigned)colscan_blocks(as)), dim3(1024), 0,
                         stream, as);
    hipLaunchKernelGGL(k_bin_scan<Real>, dim3(1), dim3(1024), 0, stream, as, tt, own_header);
    if (a.n == 0) return hipGetLastError();
    hipLaunchKernelGGL(k_scatter<Real>, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, stream,
                       a);
  }
  hipLaunchKernelGGL(k_cell_sort<Real>, dim3((unsigned)sort_blocks(a)), dim3(kSortThreads), 0,
                     stream, a, tt);
  return hipGetLastError();
}

// Sets cum[] of a batch from per-system block counts.
template <typename F>
static int64_t batch_blocks(Batch<float>& b, F per_sys) {
  b.cum[0] = 0;
  for (int s = 0; s < b.n; ++s) b.cum[s + 1] = b.cum[s] + per_sys(b.sys[s]);
  return b.cum[b.n];
}

hipError_t launch_binning_batch(const Batch<float>& b0, const TypeTable& tt, hipStream_t stream) {
  Batch<float> b = b0;
  size_t shmem = 0;
  for (int s = 0; s < b.n; ++s) {
    const size_t need = sizeof(int32_t) * (size_t)(b.sys[s].n_cells + 1);
    shmem = need > shmem ? need : shmem;
  }
  int64_t nb = batch_blocks(b, [](const SysArgs<float>& a) { return (int64_t)a.bin_blocks; });
  hipLaunchKernelGGL(k_bin_hist_batch, dim3((unsigned)nb), dim3(kBinThreads), shmem, stream, b);
  // grids of more than kScanFused cells (the others need no scan kernels)
  nb = batch_blocks(b, [](const SysArgs<float>& a) { return colscan_blocks(a); });
  if (nb > 0) hipLaunchKernelGGL(k_bin_colscan_batch, dim3((unsigned)nb), dim3(1024), 0, stream, b);
  nb = batch_blocks(b, [](const SysArgs<float>& a) { return scan_fused(a) ? (int64_t)0 : (int64_t)1; });
  if (nb > 0) {
    hipLaunchKernelGGL(k_bin_scan_batch, dim3((unsigned)nb), dim3(1024), 0, stream, b, tt);
    nb = batch_blocks(b, [](const SysArgs<float>& a) {
      return scan_fused(a) ? (int64_t)0 : (a.n + 255) / 256;
    });
    hipLaunchKernelGGL(k_scatter_batch, dim3((unsigned)nb), dim3(256), 0, stream, b);
  }
  nb = batch_blocks(b, [](const SysArgs<float>& a) { return sort_blocks(a); });
  hipLaunchKernelGGL(k_cell_sort_batch, dim3((unsigned)nb), dim3(kSortThreads), 0, stream, b, tt);
  return hipGetLastError();
}

template hipError_t launch_binning<float>(const SysArgs<float>&, const TypeTable&, hipStream_t);
template hipError_t launch_binning<double>(const SysArgs<double>&, const TypeTable&, hipStream_t);

}  // namespace md
