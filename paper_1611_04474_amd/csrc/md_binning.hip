// Cell binning: a counting sort of the atoms into cells of edge >= r_cut
// (Section 2.1, Fig. 2), stored as flat arrays instead of linked lists (the second
// code transformation of Section 2.2). Positions become a sorted structure of
// arrays (first transformation of Section 2.2): float4/double4 (x, y, z, q), the
// type and the permutation back to the caller's order.
//
// Kernels, in launch order:
//   k_setup      clears the cell counters and status word, builds the mixed
//                Lennard-Jones table (Lorentz-Berthelot) in the workspace;
//   k_bin_count  wraps each coordinate into [0, L] (one add/subtract of L in the input
//                precision), checks it, computes the cell and takes a slot with an atomic;
//   k_scan       one workgroup: exclusive prefix sum of the counts -> cell_start;
//   k_scatter    writes each atom's index at cell_start + slot (arbitrary order in a cell);
//   k_cell_sort  one workgroup per cell: orders the cell's atoms by (wrapped x, original
//                index) -- a total order, so every later sum runs in a reproducible order,
//                and a row of cells along x is sorted in x, which lets the pair kernel
//                bound each home atom's candidates by an x-window -- and writes the sorted
//                arrays.
#include "md_common.hpp"

namespace md {
namespace {

struct TypeTable {
  double sigma[kMaxTypes];
  double eps[kMaxTypes];
};

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
  return x;
}

template <typename Real>
__device__ inline int cell_coord(Real x, Real inv_w, int n) {
  int c = (int)(x * inv_w);
  c = c < 0 ? 0 : c;
  return c > n - 1 ? n - 1 : c;
}

template <typename Real>
__global__ void k_setup(SysArgs<Real> a, TypeTable tt) {
  int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t c = tid; c < a.n_cells; c += stride) a.count[c] = 0;
  if (a.flags & MD_ACCUM_F32_ATOMIC)
    for (int64_t i = tid; i < 3 * a.n; i += stride) a.facc[i] = 0.f;
  if (a.flags & MD_DIAG_COUNTERS)
    for (int64_t i = tid; i < a.n; i += stride) a.paircount[a.n + i] = 0;
  int nt = a.n_types;
  for (int64_t e = tid; e < nt * nt; e += stride) {
    int ti = (int)(e / nt), tj = (int)(e % nt);
    double s = 0.5 * (tt.sigma[ti] + tt.sigma[tj]);
    double ep = sqrt(tt.eps[ti] * tt.eps[tj]);
    double s2 = s * s, s6 = s2 * s2 * s2;
    a.lj[2 * e + 0] = (Real)(4.0 * ep * s6 * s6);
    a.lj[2 * e + 1] = (Real)(4.0 * ep * s6);
  }
  if (tid == 0) {
    a.hdr->status = 0;
    a.hdr->diag[0] = 0;
    a.hdr->diag[1] = 0;
    a.hdr->diag[2] = 0;
    a.hdr->diag[3] = 0;
  }
}

template <typename Real>
__global__ void k_bin_count(SysArgs<Real> a) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  uint32_t st = 0;
  Real x = wrap_coord(a.pos_in[3 * i + 0], a.L[0], st);
  Real y = wrap_coord(a.pos_in[3 * i + 1], a.L[1], st);
  Real z = wrap_coord(a.pos_in[3 * i + 2], a.L[2], st);
  int t = a.type_in[i];
  if (t < 0 || t >= a.n_types) st |= MD_STATUS_BAD_TYPE;
  int cx = cell_coord(x, a.inv_w[0], a.nx);
  int cy = cell_coord(y, a.inv_w[1], a.ny);
  int cz = cell_coord(z, a.inv_w[2], a.nz);
  int c = (cz * a.ny + cy) * a.nx + cx;
  a.cell[i] = c;
  a.rank[i] = atomicAdd(&a.count[c], 1);
  if (st) atomicOr(&a.hdr->status, st);
}

// Exclusive scan of count[0..n_cells) into start[], start[n_cells] = n. One
// workgroup of 1024 threads walks the array in chunks of 4096 with a running carry.
__global__ __launch_bounds__(1024) void k_scan(const int32_t* count, int32_t* start,
                                               int64_t n_cells) {
  __shared__ int32_t s[1024];
  __shared__ int32_t carry;
  int t = threadIdx.x;
  if (t == 0) carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < n_cells; base += 4096) {
    int32_t v[4];
    int32_t sum = 0;
    for (int k = 0; k < 4; ++k) {
      int64_t idx = base + 4 * t + k;
      v[k] = idx < n_cells ? count[idx] : 0;
      sum += v[k];
    }
    s[t] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {   // inclusive Hillis-Steele scan
      int32_t add = t >= off ? s[t - off] : 0;
      __syncthreads();
      s[t] += add;
      __syncthreads();
    }
    int32_t run = carry + s[t] - sum;             // exclusive prefix of this thread
    for (int k = 0; k < 4; ++k) {
      int64_t idx = base + 4 * t + k;
      if (idx < n_cells) start[idx] = run;
      run += v[k];
    }
    __syncthreads();
    if (t == 1023) carry += s[1023];
    __syncthreads();
  }
  if (t == 0) start[n_cells] = carry;
}

template <typename Real>
__global__ void k_scatter(SysArgs<Real> a) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  a.unsorted[a.start[a.cell[i]] + a.rank[i]] = (int32_t)i;
}

// One workgroup per cell. Each member's position in the cell is the number of members
// that precede it in (wrapped x, original index) order, counted over LDS chunks of the
// member list, so any cell occupancy is handled.
template <typename Real>
__global__ __launch_bounds__(256) void k_cell_sort(SysArgs<Real> a) {
  constexpr int kChunk = 1024;
  constexpr int kPer = kChunk / 256;
  __shared__ int32_t s_idx[kChunk];
  __shared__ Real s_x[kChunk];
  int64_t c = blockIdx.x;
  int32_t s0 = a.start[c];
  int32_t m = a.start[c + 1] - s0;
  for (int32_t a0 = 0; a0 < m; a0 += kChunk) {
    int32_t my_idx[kPer];
    Real my_x[kPer];
    int32_t my_rank[kPer];
    for (int k = 0; k < kPer; ++k) {
      int32_t e = a0 + (int32_t)threadIdx.x + 256 * k;
      my_idx[k] = e < m ? a.unsorted[s0 + e] : -1;
      uint32_t st = 0;
      my_x[k] = my_idx[k] >= 0 ? wrap_coord(a.pos_in[3 * (int64_t)my_idx[k]], a.L[0], st) : Real(0);
      my_rank[k] = 0;
    }
    for (int32_t b0 = 0; b0 < m; b0 += kChunk) {
      int32_t mb = min(kChunk, m - b0);
      __syncthreads();
      for (int32_t e = threadIdx.x; e < mb; e += 256) {
        const int32_t i = a.unsorted[s0 + b0 + e];
        uint32_t st = 0;
        s_idx[e] = i;
        s_x[e] = wrap_coord(a.pos_in[3 * (int64_t)i], a.L[0], st);
      }
      __syncthreads();
      for (int32_t e = 0; e < mb; ++e) {
        const int32_t v = s_idx[e];
        const Real xv = s_x[e];
        for (int k = 0; k < kPer; ++k)
          my_rank[k] += (xv < my_x[k] || (xv == my_x[k] && v < my_idx[k])) ? 1 : 0;
      }
    }
    for (int k = 0; k < kPer; ++k) {
      int32_t i = my_idx[k];
      if (i < 0) continue;
      uint32_t st = 0;
      Real x = wrap_coord(a.pos_in[3 * (int64_t)i + 0], a.L[0], st);
      Real y = wrap_coord(a.pos_in[3 * (int64_t)i + 1], a.L[1], st);
      Real z = wrap_coord(a.pos_in[3 * (int64_t)i + 2], a.L[2], st);
      int t = a.type_in[i];
      if (t < 0 || t >= a.n_types) t = 0;
      int32_t d = s0 + my_rank[k];
      P4<Real> p;
      p.x = x;
      p.y = y;
      p.z = z;
      p.w = a.q_in[i];
      a.pos[d] = p;
      a.type[d] = t;
      a.perm[d] = i;
    }
  }
}

}  // namespace

template <typename Real>
hipError_t launch_binning(const SysArgs<Real>& a, const double* sigma, const double* eps,
                          hipStream_t stream) {
  TypeTable tt;
  for (int t = 0; t < kMaxTypes; ++t) {
    tt.sigma[t] = t < a.n_types ? sigma[t] : 0.0;
    tt.eps[t] = t < a.n_types ? eps[t] : 0.0;
  }
  int64_t work = a.n_cells;
  if (a.n_types * a.n_types > work) work = a.n_types * a.n_types;
  if (3 * a.n > work) work = 3 * a.n;
  int64_t blocks = (work + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_setup<Real>, dim3((unsigned)blocks), dim3(256), 0, stream, a, tt);
  if (a.n == 0) return hipGetLastError();
  unsigned nb = (unsigned)((a.n + 255) / 256);
  hipLaunchKernelGGL(k_bin_count<Real>, dim3(nb), dim3(256), 0, stream, a);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, stream, (const int32_t*)a.count, a.start,
                     a.n_cells);
  hipLaunchKernelGGL(k_scatter<Real>, dim3(nb), dim3(256), 0, stream, a);
  hipLaunchKernelGGL(k_cell_sort<Real>, dim3((unsigned)a.n_cells), dim3(256), 0, stream, a);
  return hipGetLastError();
}

template hipError_t launch_binning<float>(const SysArgs<float>&, const double*, const double*,
                                          hipStream_t);
template hipError_t launch_binning<double>(const SysArgs<double>&, const double*,
                                           const double*, hipStream_t);

}  // namespace md
