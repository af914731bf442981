// Internal declarations shared by the translation units of the force library.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "mdforce.h"

namespace md {

constexpr int kMaxTypes = 64;
constexpr int kTasksPerCell = 14;    // predicated kernel: home cell + 13 forward neighbours
constexpr int kSlots = 27;           // partial-force slots per atom: 14 as home, 13 as neighbour
constexpr int kTile = 256;           // atoms of one cell staged in LDS at a time
constexpr int kPairThreads = 256;    // threads of one predicated pair workgroup (4 waves)
constexpr int64_t kMaxCells = 1 << 24;
constexpr int64_t kMaxAtoms = (int64_t)1 << 30;
constexpr int kBinLdsCells = 32768;  // largest grid binned with a per-block LDS histogram
constexpr int kBinMaxBlocks = 1024;  // blocks of that pass
constexpr int kBinThreads = 512;     // threads per block of that pass
constexpr int kBinChunkUnit = 2048;  // atoms per block: a multiple of this (4 per thread)
// A^2 added to rc^2 by the compacted kernel's expanded-form prefilter (its constants per
// home atom are written by the in-cell sort)
constexpr float kPrefilterMargin = 0.05f;

// Workspace header (first 256 bytes).
// Drain depth selected by MD_PAIR_DRAIN in md_params.flags (2 when the field is 0).
__host__ __device__ inline int md_pair_drain(uint32_t flags) {
  const uint32_t v = (flags & MD_PAIR_DRAIN_MASK) >> 5;
  return v == 0 ? 2 : v == 1 ? 1 : v == 2 ? 3 : 4;
}

// Workgroups of the compacted pair kernel per home cell, each taking every split-th group
// of the cell's home atoms: MD_PAIR_SPLIT(s) in md_params.flags, or (field 0) automatic:
// grids of fewer than 128 (4) or 64 (2) cells take 2 or 4, so that the 256 compute units get
// work; larger grids take 1 (a split repeats the staging and the neighbour-side flush, which
// measured 25% slower at 486 cells).
__host__ __device__ inline int md_fs_split(uint32_t flags, int64_t n_cells) {
  const uint32_t v = (flags & MD_PAIR_SPLIT_MASK) >> 8;
  if (v) return v == 1 ? 1 : v == 2 ? 2 : 4;
  if (n_cells <= 0) return 1;
  const int64_t s = 256 / n_cells;   // workgroups per compute unit's worth of cells
  return s >= 4 ? 4 : s >= 2 ? 2 : 1;
}

struct WsHeader {
  uint32_t status;
  uint32_t pad0;
  unsigned long long diag[5];   // candidates, filter passes, cutoff passes, filtered slots,
                                // force lanes evaluated
  unsigned long long clock[2];  // compacted pair kernel since the last binning, summed over
                                // its workgroups: shader-clock cycles, 100 MHz ticks
  uint32_t cost_key;            // kCostKey when cost[] holds the last pair kernel's times
  uint32_t cost_cells;          // ... of a grid of this many cells
  uint32_t pad1[46];
};
constexpr uint32_t kCostKey = 0x4d44434fu;
static_assert(sizeof(WsHeader) == 256, "header size");

// An atom's in-cell sort key and type, written by the scatter with one 16-byte store.
struct alignas(16) UKey {
  unsigned long long key;
  int32_t type;
  int32_t pad;
};

template <typename Real>
struct alignas(4 * sizeof(Real)) P4 {
  Real x, y, z, w;
};

// A small non-negative integer carried in a Real slot as bits (no arithmetic is done on it).
template <typename Real>
__device__ inline Real int_to_slot(int32_t v) {
  if constexpr (sizeof(Real) == 4) return __int_as_float(v);
  else return __longlong_as_double((long long)v);
}
template <typename Real>
__device__ inline int32_t slot_to_int(Real v) {
  if constexpr (sizeof(Real) == 4) return __float_as_int(v);
  else return (int32_t)__double_as_longlong(v);
}

// Cell grid and workspace carve-up for one system.
struct Plan {
  int32_t dims[3];
  int64_t n_cells;
  int64_t n_tasks;
  int64_t n;
  int real_bytes;               // 4 or 8
  // byte offsets
  size_t off_count, off_start, off_cell, off_rank, off_pos, off_hpre, off_type, off_perm,
      off_part, off_facc, off_epart, off_lj, off_paircount, off_bhist, off_bstat, off_order,
      off_cost,
      off_zsplit, off_ukey, off_upos, off_kpart, total;
  int bin_blocks;               // blocks of the LDS-histogram binning pass (0: global atomics)
  int64_t bin_chunk;            // atoms per such block
};

// Computes the grid and workspace layout; returns MD_OK or an error code.
md_status make_plan(const md_params* p, int64_t n, int real_bytes, Plan* out);

// Kernel-side constants of one system.
template <typename Real>
struct SysArgs {
  // inputs
  const Real* pos_in;          // [n][3]
  const int32_t* type_in;      // [n]
  const Real* q_in;            // [n]
  Real* force_out;             // [n][3]
  double* energy_out;          // [1]
  // workspace
  WsHeader* hdr;
  int32_t* count;              // [n_cells]
  int32_t* start;              // [n_cells+1]
  int32_t* cell;               // [n]
  int32_t* rank;               // [n] (also the in-cell sort's member list of a cell of more
                               // than 1024 atoms, with the fused scan)
  UKey* ukey;                  // [n] in-cell sort keys and types, in cell order before the
                               // in-cell sort (with the fused scan: in cell order within
                               // each histogram block's range)
  P4<Real>* upos;              // [n] wrapped (x, y, z, q), same order
  P4<Real>* pos;               // [n] sorted (x,y,z,q)
  P4<Real>* hpre;              // [2n] sorted, for the compacted kernel (written by the
                               // in-cell sort): the atom's prefilter constants as a home
                               // atom, (ax, ay, az, thb) = (-2 a, rc^2 + margin - |a|^2 -
                               // 2 a.o) with a = r - o, o its cell's centre, and
                               // (k q, type n_types as integer bits, 0, 0)
  int32_t* type;               // [n] sorted
  int32_t* perm;               // [n] sorted -> original
  Real* part;                  // [kSlots][3][n]
  float* facc;                 // [3][n]
  double* epart;               // [n_tasks]
  Real* lj;                    // [n_types^2][2] (c12, c6)
  int32_t* paircount;          // [2][n]: caller order (after finalize), sorted order (pass)
  long long* acc64;            // per-atom fixed-point sums of the compacted kernel: float32
                               // [3][n] (2^-28 kcal/mol/A); float64 [2][3][n], the high
                               // words (2^-20) then the low words (2^-72)
  int32_t* bhist;              // grids of at most 1024 cells: [bin_blocks][n_cells + 1] each
                               // block's start of every cell within its range (then its
                               // atom count); larger grids: [bin_blocks][n_cells] per-block
                               // cell counts (offsets in place after k_bin_colscan)
  uint32_t* bstat;             // [bin_blocks] per-block status bits
  int32_t* order;              // [n_cells] launch order of the home cells, longest first
  uint32_t* cost;              // [n_cells] each home cell's time in the last pair kernel
  int32_t* zsplit;             // [n_cells] atoms of each cell in its lower z half
  // scalars
  int64_t n, n_cells, n_tasks;
  int bin_blocks;
  int64_t bin_chunk;
  int nx, ny, nz, n_types;
  Real L[3];                   // box (rounded once to Real)
  Real inv_w[3];               // n_d / L_d
  Real rc2, rs2, inv_sw;       // inv_sw = 1/(rc2 - rs2), 0 when switching is off
  Real coulomb_k;
  Real ewald_alpha;            // 1/A, with MD_COULOMB_EWALD (0 otherwise)
  uint32_t flags;
  int compact;                 // 1: per-atom sums come from the compacted pair kernel (acc64,
                               //    or, float32 only, facc with MD_ACCUM_F32_ATOMIC)
  int half_shell;              // 1: the compacted kernel visits each pair once and adds
                               //    into acc64 with integer atomics (acc64 starts at zero)
  int fs_split;                // compacted-kernel workgroups per home cell (md_fs_split)
};

// Up to kBatchMax systems evaluated by one launch of each kernel of the path. The
// systems' arguments travel in the kernel argument block; block b of a batched launch
// belongs to system s with cum[s] <= b < cum[s+1], as its local block b - cum[s].
constexpr int kBatchMax = 10;   // keeps every batched kernel's arguments under 4 KB

template <typename Real>
struct Batch {
  int n;
  int64_t cum[kBatchMax + 1];
  SysArgs<Real> sys[kBatchMax];

  __device__ inline int pick(int64_t b, int64_t& local) const {
    int s = 0;
    while (s + 1 < n && cum[s + 1] <= b) ++s;
    local = b - cum[s];
    return s;
  }
};

// Per-type sigma and epsilon, mixed into the LJ table by the binning stage.
struct TypeTable {
  double sigma[kMaxTypes];
  double eps[kMaxTypes];
};

template <typename Real>
SysArgs<Real> make_args(const md_params* p, const Plan& pl, int64_t n, const Real* pos,
                        const int32_t* type, const Real* q, Real* force, double* energy,
                        void* ws);

// Launchers (each enqueues on `stream`, returns hipSuccess or an error).
TypeTable make_type_table(const md_params* p);
template <typename Real>
hipError_t launch_binning(const SysArgs<Real>& a, const TypeTable& tt, hipStream_t stream);
template <typename Real>
hipError_t launch_pair(const SysArgs<Real>& a, hipStream_t stream);
template <typename Real>
hipError_t launch_finalize(const SysArgs<Real>& a, hipStream_t stream);
template <typename Real>
hipError_t launch_pair_fs(const SysArgs<Real>& a, hipStream_t stream);

// Batched float32 launchers. Every system of the batch has n > 0, uses the LDS-histogram
// binning (bin_blocks > 0), the compacted kernel, and the same flags and
// type table.
hipError_t launch_binning_batch(const Batch<float>& b, const TypeTable& tt, hipStream_t stream);
hipError_t launch_pair_fs_batch(const Batch<float>& b, hipStream_t stream);
hipError_t launch_finalize_batch(const Batch<float>& b, hipStream_t stream);

// Velocity-Verlet kernels of md_run_vv_f32 (md_integrate.hip). kick_drift: v += h F/m,
// x += dt v wrapped into [0, L). kick: v += h F/m, and the kinetic energy, from per-block
// partials in kpart ([ke_blocks(n)] doubles) summed in a fixed order into *ke.
int64_t ke_blocks(int64_t n);
hipError_t launch_vv_kick_drift(int64_t n, float* pos, float* vel, const float* force,
                                const float* inv_mass, float h, float dt, const float* L,
                                hipStream_t stream);
hipError_t launch_vv_kick(int64_t n, float* vel, const float* force, const float* inv_mass,
                          float h, double* kpart, double* ke, hipStream_t stream);

}  // namespace md
