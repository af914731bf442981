// Finalize: per-atom force sums and the total energy.
//
// k_finalize writes each sorted atom's force in the caller's atom order. After the
// compacted kernel it converts the per-atom fixed-point sums to float: float32 from one
// 64-bit word (2^-28 kcal/mol/A), float64 from two (hi 2^-20 + lo 2^-72). After the
// predicated kernel it adds the 27 partial forces of the atom (14 as a home atom, 13 as a
// neighbour): in float32 converted to 64-bit fixed point (one unit = 2^-32 kcal/mol/A,
// round to nearest even) and summed as integers, so the per-atom total does not depend on
// any summation order (an out-of-range value sets MD_STATUS_FIXED_OVERFLOW); in float64
// in slot order.
//
// The energy block adds the per-workgroup float64 energy partials in a fixed tree order;
// it is one more block of the same launch.
#include "md_common.hpp"

namespace md {
namespace {

__device__ inline float fixed_sum(const float* part, int64_t n, int c, int64_t s, uint32_t& st) {
  const double kScale = 4294967296.0;       // 2^32
  const double kLimit = 9.2233720368547e18; // 2^63
  long long acc = 0;
  for (int slot = 0; slot < kSlots; ++slot) {
    float v = part[((int64_t)slot * 3 + c) * n + s];
    double d = (double)v * kScale;          // exact: 24-bit significand, power-of-two scale
    if (!(fabs(d) < kLimit)) {
      st |= MD_STATUS_FIXED_OVERFLOW;
      continue;
    }
    long long q = __double2ll_rn(d);
    long long r;
    if (__builtin_add_overflow(acc, q, &r)) {
      st |= MD_STATUS_FIXED_OVERFLOW;
      continue;
    }
    acc = r;
  }
  return __ll2float_rn(acc) * 2.3283064365386963e-10f;   // * 2^-32, exact
}

template <typename Real>
__device__ inline void finalize(const SysArgs<Real>& a, int64_t blk) {
  int64_t s = blk * 256 + threadIdx.x;
  if (s >= a.n) return;
  const int64_t i = a.perm[s];
  uint32_t st = 0;
  Real f[3];
  for (int c = 0; c < 3; ++c) {
    Real v;
    if (a.flags & MD_ACCUM_F32_ATOMIC) {
      v = (Real)a.facc[(int64_t)c * a.n + s];
    } else if (a.compact && sizeof(Real) == 4) {
      v = (Real)(__ll2float_rn(a.acc64[(int64_t)c * a.n + s]) * 3.725290298461914e-09f);   // 2^-28
    } else if (a.compact) {
      // two-word sum: hi 2^-20 + lo 2^-72 (hi exact in float64, one rounding of lo, one of
      // the sum)
      v = (Real)((double)a.acc64[(int64_t)c * a.n + s] * 9.5367431640625e-07 +
                 (double)a.acc64[(int64_t)(3 + c) * a.n + s] * 2.117582368135751e-22);
    } else if (sizeof(Real) == 4) {
      v = (Real)fixed_sum(reinterpret_cast<const float*>(a.part), a.n, c, s, st);
    } else {
      Real acc = 0;
      for (int slot = 0; slot < kSlots; ++slot) acc += a.part[((int64_t)slot * 3 + c) * a.n + s];
      v = acc;
    }
    f[c] = v;
  }
  // one store of the three components
  struct alignas(sizeof(Real)) R3 {
    Real x, y, z;
  };
  *reinterpret_cast<R3*>(a.force_out + 3 * i) = R3{f[0], f[1], f[2]};
  if (a.flags & MD_DIAG_COUNTERS) a.paircount[i] = a.paircount[a.n + s];
  if (st) atomicOr(&a.hdr->status, st);
}

__device__ inline void energy(const double* epart, int64_t n_tasks, double* out, WsHeader* hdr,
                              int halve_diag) {
  if (halve_diag && threadIdx.x < 5) hdr->diag[threadIdx.x] /= 2;
  __shared__ double s[256];
  double acc = 0.0;
  // each thread adds its partials in index order, eight loads in flight at a time
  for (int64_t t0 = threadIdx.x; t0 < n_tasks; t0 += 8 * 256) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t t = t0 + 256 * u;
      v[u] = t < n_tasks ? epart[t] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (t0 + 256 * u < n_tasks) acc += v[u];
  }
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = s[0];
}

template <typename Real>
__host__ __device__ inline int64_t energy_parts(const SysArgs<Real>& a) {
  return a.n > 0 ? (a.compact ? a.n_cells * a.fs_split : a.n_tasks) : 0;
}

template <typename Real>
__host__ __device__ inline int halve_diag(const SysArgs<Real>& a) {
  return (a.compact && !a.half_shell && (a.flags & MD_DIAG_COUNTERS) && a.n > 0) ? 1 : 0;
}

// Energy after the compacted kernel: its workgroups' exact integer sums (float32: one int64
// in units of 2^-24 kcal/mol; float64: two words, hi 2^-20 + lo 2^-72, lo in [0, 2^52)),
// added as integers in a fixed order, so the total is the same bits however the work was
// split into workgroups; the full shell saw every pair twice (factor 1/2, exact).
template <typename Real>
__device__ inline void energy_fixed(const SysArgs<Real>& a, int64_t n_parts) {
  if (halve_diag(a) && threadIdx.x < 5) a.hdr->diag[threadIdx.x] /= 2;
  __shared__ long long s_hi[256], s_lo[256];
  const long long* ep = reinterpret_cast<const long long*>(a.epart);
  constexpr bool f64 = sizeof(Real) == 8;
  long long hi = 0, lo = 0;
  for (int64_t t = threadIdx.x; t < n_parts; t += 256) {
    if (f64) {
      hi += ep[2 * t];
      lo += ep[2 * t + 1];
      hi += lo >> 52;   // carry: lo stays in [0, 2^52)
      lo &= (1ll << 52) - 1;
    } else {
      hi += ep[t];
    }
  }
  s_hi[threadIdx.x] = hi;
  s_lo[threadIdx.x] = lo;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      long long h = s_hi[threadIdx.x] + s_hi[threadIdx.x + off];
      long long l = s_lo[threadIdx.x] + s_lo[threadIdx.x + off];
      s_hi[threadIdx.x] = h + (l >> 52);
      s_lo[threadIdx.x] = l & ((1ll << 52) - 1);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double f = a.half_shell ? 1.0 : 0.5;
    *a.energy_out = f64 ? f * ((double)s_hi[0] * 9.5367431640625e-07 + (double)s_lo[0] * 2.117582368135751e-22)
                        : f * ((double)s_hi[0] * 5.9604644775390625e-08);   // 2^-20, 2^-72; 2^-24
  }
}

// Block 0 sums the energy partials, which the pair kernel has completed, and blocks
// 1 .. ceil(n/256) finalize atoms, so one launch does both; the energy block, the longest,
// is dispatched first.
template <typename Real>
__device__ inline void finalize_or_energy(const SysArgs<Real>& a, int64_t blk) {
  if (blk == 0) {
    if (a.compact)
      energy_fixed(a, energy_parts(a));
    else
      energy(a.epart, energy_parts(a), a.energy_out, a.hdr, halve_diag(a));
    return;
  }
  finalize(a, blk - 1);
}

template <typename Real>
__global__ __launch_bounds__(256) void k_finalize_energy(SysArgs<Real> a) {
  finalize_or_energy(a, blockIdx.x);
}

__global__ __launch_bounds__(256) void k_finalize_energy_batch(Batch<float> b) {
  int64_t blk;
  const int s = b.pick(blockIdx.x, blk);
  finalize_or_energy(b.sys[s], blk);
}

}  // namespace

template <typename Real>
hipError_t launch_finalize(const SysArgs<Real>& a, hipStream_t stream) {
  const unsigned nb = (unsigned)((a.n + 255) / 256) + 1;
  hipLaunchKernelGGL(k_finalize_energy<Real>, dim3(nb), dim3(256), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_finalize_batch(const Batch<float>& b0, hipStream_t stream) {
  Batch<float> b = b0;
  b.cum[0] = 0;
  for (int s = 0; s < b.n; ++s) b.cum[s + 1] = b.cum[s] + (b.sys[s].n + 255) / 256 + 1;
  hipLaunchKernelGGL(k_finalize_energy_batch, dim3((unsigned)b.cum[b.n]), dim3(256), 0, stream, b);
  return hipGetLastError();
}

template hipError_t launch_finalize<float>(const SysArgs<float>&, hipStream_t);
template hipError_t launch_finalize<double>(const SysArgs<double>&, hipStream_t);

}  // namespace md
