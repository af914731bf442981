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
// then, for grids of at most 1024 cells,
//   k_scatter_fused  every block derives the cells' starts and its own offset within each
//                    cell from the histograms and scatters its atoms; block 0 also writes
//                    cell_start, the launch order, the mixed Lennard-Jones table
//                    (Lorentz-Berthelot) and the status word;
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
//                    and the number of atoms in the lower z half.
// The scatter puts atoms in arbitrary order within a cell's range (the LDS atomics' order);
// the launch order puts the cells longest first (atom counts, or the last pair kernel's
// measured times on small grids), so that the last workgroups to run are short ones.
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

template <typename Real>
__device__ inline void bin_hist(const SysArgs<Real>& a, int64_t blk) {
  extern __shared__ int32_t s_h[];   // [n_cells] counts, then the status bits
  const int nc = (int)a.n_cells;
  const int tid = threadIdx.x;
  for (int c = tid; c <= nc; c += kBinThreads) s_h[c] = 0;
  __syncthreads();
  const int64_t i0 = blk * a.bin_chunk;
  const int64_t i1 = i0 + a.bin_chunk < a.n ? i0 + a.bin_chunk : a.n;
  uint32_t st = 0;
  for (int64_t r0 = i0; r0 < i1; r0 += kBinThreads * kHistPer) {
    Real x[kHistPer], y[kHistPer], z[kHistPer];
    int ty[kHistPer], c[kHistPer];
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
    }
#pragma unroll
    for (int u = 0; u < kHistPer; ++u) c[u] = cell_from(a, x[u], y[u], z[u], ty[u], st);
#pragma unroll
    for (int u = 0; u < kHistPer; ++u) {
      const int64_t i = r0 + u * kBinThreads + tid;
      if (i < i1) {
        a.cell[i] = c[u];
        a.rank[i] = atomicAdd(&s_h[c[u]], 1);
        clear_atom(a, i);
      }
    }
  }
  if (st) atomicOr(reinterpret_cast<uint32_t*>(&s_h[nc]), st);
  __syncthreads();
  int32_t* hb = a.bhist + blk * nc;
  for (int c = tid; c < nc; c += kBinThreads) hb[c] = s_h[c];
  if (tid == 0) a.bstat[blk] = (uint32_t)s_h[nc];
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

// Exclusive prefix sum of one value per thread over a 1024-thread workgroup: a scan
// within each wave, then the 16 wave totals through LDS. *total gets the sum of all.
__device__ inline int32_t block_scan_excl(int32_t v, int32_t* s_tot, int32_t* total) {
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
  for (int k = 0; k < 16; ++k) {
    const int32_t tk = s_tot[k];
    before += k < w ? tk : 0;
    all += tk;
  }
  __syncthreads();   // s_tot may be reused after this
  *total = all;
  return before + x - v;
}

// Grids of at most kScanFused cells binned with per-block histograms skip the scan
// kernels: every block of k_scatter_fused scans the histograms itself (one thread per
// cell). Larger grids go through k_bin_colscan, k_bin_scan and k_scatter.
constexpr int kScanFused = 1024;

template <typename Real>
__host__ __device__ inline bool scan_fused(const SysArgs<Real>& a) {
  return a.bin_blocks > 0 && a.n_cells <= kScanFused;
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
// status word: the end of the scan, by one workgroup of 1024 threads. key(c) is cell c's
// expected cost: its atom count, or (grids of at most kScanFused cells) its time in the
// last pair kernel when known; st_lane (threads 0 .. 63) carries the histogram blocks'
// status bits from block_status.
template <typename Real, typename Key>
__device__ inline void scan_tail(const SysArgs<Real>& a, const TypeTable& tt, int own_header,
                                 int32_t* s_tot, Key key, uint32_t st_lane) {
  const int t = threadIdx.x;
  const int64_t nc = a.n_cells;
  // counting sort of the cells by decreasing key (keys clamped to kOrderBins - 1); the
  // order within a bin is arbitrary, which only changes which compute unit takes a cell,
  // never a result. Longest first lets the short cells fill the tail.
  constexpr int kOrderBins = 1024;
  __shared__ int32_t s_bin[kOrderBins];
  s_bin[t] = 0;
  __syncthreads();
  auto bin = [&](int64_t c) {
    const uint32_t v = key(c);
    return kOrderBins - 1 - (int)(v < kOrderBins - 1 ? v : kOrderBins - 1);
  };
  for (int64_t c = t; c < nc; c += 1024) atomicAdd(&s_bin[bin(c)], 1);
  __syncthreads();
  {
    int32_t all;
    const int32_t excl = block_scan_excl(s_bin[t], s_tot, &all);
    s_bin[t] = excl;   // each thread rewrites only its own bin, read above
    __syncthreads();
  }
  for (int64_t c = t; c < nc; c += 1024) {
    const int32_t pos = atomicAdd(&s_bin[bin(c)], 1);
    a.order[pos] = (int32_t)c;
  }
  const int nt = a.n_types;
  for (int e = t; e < nt * nt; e += 1024) {
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
  scan_tail(a, tt, own_header, s_tot, [&](int64_t c) { return (uint32_t)count(c); },
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

// Atom i (of cell c) goes to slot `slot` of the cell-major arrays that precede the in-cell
// sort: its sort key and type as one 16-byte record, and its wrapped (x, y, z, q).
template <typename Real>
__device__ inline void put_atom(const SysArgs<Real>& a, int64_t i, int c, int32_t slot, Real x,
                                Real y, Real z, Real q, int t) {
  const int cz = (int)(c / ((int64_t)a.nx * a.ny));
  uint32_t st = 0;
  P4<Real> p;
  p.x = wrap_coord(x, a.L[0], st);
  p.y = wrap_coord(y, a.L[1], st);
  p.z = wrap_coord(z, a.L[2], st);
  p.w = q;
  if (t < 0 || t >= a.n_types) t = 0;
  a.ukey[slot] = UKey{sort_key(a, (int32_t)i, (float)p.x, p.z, cz), t, 0};
  a.upos[slot] = p;
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
  put_atom(a, i, c, slot, a.pos_in[3 * i + 0], a.pos_in[3 * i + 1], a.pos_in[3 * i + 2],
           a.q_in[i], a.type_in[i]);
}

// Grids of at most kScanFused cells with per-block histograms: block blk (1024 threads)
// takes atoms 1024 blk .. 1024 blk + 1023, which lie in histogram block
// hb = 1024 blk / bin_chunk. Thread c adds up the histogram blocks' counts of cell c, all
// of them and those of the blocks before hb; the totals are scanned into the cells' starts
// in LDS, and each atom goes to start[c] + (offset of block hb in cell c) + (its rank
// within hb). Every block repeats this scan, which replaces a kernel of its own; one more
// block, the last, scatters nothing: it writes start[] and runs scan_tail, alongside the
// others. All loads are issued before the first is used.
template <typename Real>
__host__ __device__ inline int64_t fused_blocks(const SysArgs<Real>& a) {
  return scan_fused(a) ? (a.n + 1023) / 1024 + 1 : 0;
}

template <typename Real>
__device__ inline void scatter_fused(const SysArgs<Real>& a, const TypeTable& tt, int64_t blk) {
  static_assert(kScanFused <= 1024, "one cell per thread");
  static_assert(kBinChunkUnit % 1024 == 0, "a block's atoms lie in one histogram block");
  __shared__ int32_t s_tot[16];
  __shared__ int32_t s_start[kScanFused];
  __shared__ int32_t s_off[kScanFused];
  __shared__ int32_t s_cnt[kScanFused];
  const int t = threadIdx.x;
  const int nc = (int)a.n_cells;
  const int B = a.bin_blocks;
  const int64_t i = blk * 1024 + t;
  const int64_t hb = blk * 1024 / a.bin_chunk;
  // this thread's atom (a repeat of the last one past the end: nothing is stored for it)
  const int64_t ic = i < a.n ? i : a.n - 1;
  const int ci = a.cell[ic], rk = a.rank[ic];
  const Real x = a.pos_in[3 * ic + 0], y = a.pos_in[3 * ic + 1], z = a.pos_in[3 * ic + 2];
  const Real q = a.q_in[ic];
  const int ty = a.type_in[ic];
  const bool tail = blk == (a.n + 1023) / 1024;   // the block that ends the scan
  const Status st_blocks = block_status(a, tail);
  // tail block: this cell's cost in the last pair kernel (loaded before it is known whether
  // the costs are valid, so that both loads are in flight together)
  const uint32_t cost_t = tail && t < nc ? a.cost[t] : 0u;
  const bool by_cost = tail && have_costs(a);
  int32_t tot = 0, off = 0;
  if (t < nc) {
    for (int b0 = 0; b0 < B; b0 += 64) {
      int32_t v[64];
#pragma unroll
      for (int r = 0; r < 64; ++r) v[r] = b0 + r < B ? a.bhist[(int64_t)(b0 + r) * nc + t] : 0;
#pragma unroll
      for (int r = 0; r < 64; ++r) {
        tot += v[r];
        off += b0 + r < hb ? v[r] : 0;
      }
    }
  }
  int32_t all;
  const int32_t start_c = block_scan_excl(tot, s_tot, &all);
  if (t < nc) {
    s_start[t] = start_c;
    s_off[t] = off;
    s_cnt[t] = by_cost ? (int32_t)cost_key(cost_t) : tot;   // the tail block's order key
  }
  __syncthreads();
  if (i < a.n) put_atom(a, i, ci, s_start[ci] + s_off[ci] + rk, x, y, z, q, ty);
  if (tail) {
    if (t < nc) a.start[t] = start_c;
    if (t == 0) a.start[nc] = all;
    scan_tail(a, tt, 1, s_tot, [&](int64_t cc) { return (uint32_t)s_cnt[cc]; }, st_blocks.bits());
  }
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

template <typename Real>
__global__ __launch_bounds__(1024) void k_scatter_fused(SysArgs<Real> a, TypeTable tt) {
  scatter_fused(a, tt, blockIdx.x);
}

__global__ __launch_bounds__(1024) void k_scatter_fused_batch(Batch<float> b, TypeTable tt) {
  int64_t blk;
  const int s = b.pick(blockIdx.x, blk);
  scatter_fused(b.sys[s], tt, blk);
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
template <typename Real>
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
  a.hpre[2 * (int64_t)d] = h0;
  a.hpre[2 * (int64_t)d + 1] = h1;
}

template <typename Real>
__device__ inline void cell_sort(const SysArgs<Real>& a, int64_t c) {
  constexpr int kChunk = 1024;
  constexpr int kPer = kChunk / 256;
  __shared__ unsigned long long s_key[kChunk];
  __shared__ int32_t s_low;
  const int32_t s0 = a.start[c];
  const int32_t m = a.start[c + 1] - s0;
  const P4<Real> o = cell_centre(a, c);
  if (threadIdx.x == 0) s_low = 0;
  if (m == 0) {
    if (threadIdx.x == 0) a.zsplit[c] = 0;
    return;
  }
  if (m <= kChunk) {
    // the whole cell in one LDS chunk: each member's key, position and type are loaded
    // once, together, and the keys go to LDS from registers
    const int kk = (m + 255) / 256;   // member slots in use (uniform)
    unsigned long long my_key[kPer];
    Real px[kPer], py[kPer], pz[kPer], pq[kPer];
    int32_t my_t[kPer], my_rank[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int32_t e = (int32_t)threadIdx.x + 256 * k;
      const bool in = k < kk && e < m;
      const int32_t src = s0 + (in ? e : 0);   // m >= 1 here: a valid member
      const UKey u = a.ukey[src];
      my_key[k] = in ? u.key : ~0ull;
      const P4<Real> p = a.upos[src];
      px[k] = p.x;
      py[k] = p.y;
      pz[k] = p.z;
      pq[k] = p.w;
      my_t[k] = u.type;
      my_rank[k] = 0;
    }
    // slots m .. 256 kk - 1 (a multiple of 8) hold ~0, which is below no key
#pragma unroll
    for (int k = 0; k < kPer; ++k)
      if (k < kk) s_key[threadIdx.x + 256 * k] = my_key[k];
    __syncthreads();
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
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int32_t e = (int32_t)threadIdx.x + 256 * k;
      const bool in = k < kk && e < m;
      count_low(&s_low, in && !(my_key[k] >> 63));
      if (!in) continue;
      const int32_t d = s0 + my_rank[k];
      P4<Real> p;
      p.x = px[k];
      p.y = py[k];
      p.z = pz[k];
      p.w = pq[k];
      a.pos[d] = p;
      a.type[d] = my_t[k];
      a.perm[d] = (int32_t)(my_key[k] & 0x7fffffffull);
      if (a.compact) write_hpre(a, o, d, p, my_t[k]);
    }
    __syncthreads();
    if (threadIdx.x == 0) a.zsplit[c] = s_low;
    return;
  }
  for (int32_t a0 = 0; a0 < m; a0 += kChunk) {
    const int kk = min(kPer, (m - a0 + 255) / 256);   // member slots in use (uniform)
    unsigned long long my_key[kPer];
    int32_t my_rank[kPer];
    for (int k = 0; k < kPer; ++k) {
      const int32_t e = a0 + (int32_t)threadIdx.x + 256 * k;
      my_key[k] = (k < kk && e < m) ? a.ukey[s0 + e].key : ~0ull;
      my_rank[k] = 0;
    }
    for (int32_t b0 = 0; b0 < m; b0 += kChunk) {
      const int32_t mb = min(kChunk, m - b0);
      __syncthreads();
      for (int32_t e = threadIdx.x; e < mb; e += 256) s_key[e] = a.ukey[s0 + b0 + e].key;
      for (int32_t e = mb + (int32_t)threadIdx.x; e < ((mb + 3) & ~3); e += 256) s_key[e] = ~0ull;
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
      const int32_t e = a0 + (int32_t)threadIdx.x + 256 * k;
      const bool in = k < kk && e < m;
      count_low(&s_low, in && !(my_key[k] >> 63));
      if (!in) continue;
      const int32_t d = s0 + my_rank[k];
      const P4<Real> p = a.upos[s0 + e];
      const int32_t ty = a.ukey[s0 + e].type;
      a.pos[d] = p;
      a.type[d] = ty;
      a.perm[d] = (int32_t)(my_key[k] & 0x7fffffffull);
      if (a.compact) write_hpre(a, o, d, p, ty);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) a.zsplit[c] = s_low;
}

template <typename Real>
__global__ __launch_bounds__(256) void k_cell_sort(SysArgs<Real> a) { cell_sort(a, blockIdx.x); }

__global__ __launch_bounds__(256) void k_cell_sort_batch(Batch<float> b) {
  int64_t blk;
  const int s = b.pick(blockIdx.x, blk);
  cell_sort(b.sys[s], blk);
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
  if (scan_fused(as)) {
    hipLaunchKernelGGL(k_scatter_fused<Real>, dim3((unsigned)fused_blocks(as)), dim3(1024), 0,
                       stream, as, tt);
  } else {
    if (colscan_blocks(as) > 0)
      hipLaunchKernelGGL(k_bin_colscan<Real>, dim3((unsigned)colscan_blocks(as)), dim3(1024), 0,
                         stream, as);
    hipLaunchKernelGGL(k_bin_scan<Real>, dim3(1), dim3(1024), 0, stream, as, tt, own_header);
    if (a.n == 0) return hipGetLastError();
    hipLaunchKernelGGL(k_scatter<Real>, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, stream,
                       a);
  }
  hipLaunchKernelGGL(k_cell_sort<Real>, dim3((unsigned)a.n_cells), dim3(256), 0, stream, a);
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
  // grids of at most kScanFused cells: scan and scatter in one kernel
  nb = batch_blocks(b, [](const SysArgs<float>& a) { return fused_blocks(a); });
  if (nb > 0) hipLaunchKernelGGL(k_scatter_fused_batch, dim3((unsigned)nb), dim3(1024), 0, stream, b, tt);
  // larger grids
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
  nb = batch_blocks(b, [](const SysArgs<float>& a) { return a.n_cells; });
  hipLaunchKernelGGL(k_cell_sort_batch, dim3((unsigned)nb), dim3(256), 0, stream, b);
  return hipGetLastError();
}

template hipError_t launch_binning<float>(const SysArgs<float>&, const TypeTable&, hipStream_t);
template hipError_t launch_binning<double>(const SysArgs<double>&, const TypeTable&, hipStream_t);

}  // namespace md
