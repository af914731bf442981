// Pair kernel: the force stage of one iteration of the short-range non-bonded
// calculation (Algorithm 1, Section 2.1) over the half shell of cell pairs.
//
// Work unit ("task"): a home cell A and one of 14 partner images B: A itself, or one
// of the 13 forward neighbours o (lexicographically positive offsets in {-1,0,1}^3).
// Each unordered periodic image pair of cells is visited exactly once, so each pair
// of atoms within the cutoff is evaluated once and its force is applied to both
// atoms (Newton's third law). When A+o leaves the grid the image of B is shifted by
// one box length; the shift is applied exactly by subtracting L from whichever side
// lies in the last cell of that axis (Sterbenz: both operands within a factor of 2),
// so each displacement component carries a single rounding.
//
// Per task, the partial force on each atom of A is written to slot k (k = task index
// 0..13) and on each atom of B to slot 13+k of a [27][3][n] buffer. Every (slot, atom)
// is owned by exactly one task, so no atomics touch global memory and every sum runs
// in a fixed order; the finalize kernel adds the 27 partials of an atom in 64-bit
// fixed point.
//
// This is the predicated data flow: one home atom per lane; the lane walks the
// neighbour tile and evaluates the force under the cutoff predicate, so lanes whose
// candidate fails idle through the force arithmetic -- the conditional data flow that
// leaves the force unit of the HLS design underused (Section 5.1). It serves the
// MD_PAIR_PREDICATED comparison with the compacted kernel, in float32 and in float64, and
// float64 with per-atom float32 atomics (MD_ACCUM_F32_ATOMIC).
#include "md_common.hpp"

namespace md {
namespace {

// Forward offsets; index 0 is the home cell.
__constant__ int8_t c_off[kTasksPerCell][3] = {
    {0, 0, 0},   {1, 0, 0},  {-1, 1, 0}, {0, 1, 0},  {1, 1, 0},
    {-1, -1, 1}, {0, -1, 1}, {1, -1, 1}, {-1, 0, 1}, {0, 0, 1},
    {1, 0, 1},   {-1, 1, 1}, {0, 1, 1},  {1, 1, 1}};

template <typename Real>
struct Consts {
  Real rc2, rs2, inv_sw, sw12;   // sw12 = 12 * inv_sw
};

// u = dx^2 + dy^2 + dz^2. In float64 the products and sums are rounded separately,
// in the order ((dx^2 + dy^2) + dz^2), so the cutoff test decides exactly like a
// plain double evaluation of the same expression.
__device__ inline float dist2(float dx, float dy, float dz) {
  return fmaf(dz, dz, fmaf(dy, dy, dx * dx));
}
__device__ inline double dist2(double dx, double dy, double dz) {
  return __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
}

__device__ inline float rsqrt_r(float u) { return __builtin_amdgcn_rsqf(u); }
__device__ inline double rsqrt_r(double u) { return 1.0 / sqrt(u); }

// Scalar force and energy of one pair at squared distance u < rc2:
// F_i = f (x_i - x_j). Eq. 1 and Eq. 2 give f_LJ = (12 c12/r^12 - 6 c6/r^6)/u and
// f_C = k qi qj / r / u; the switch S(u) multiplies the pair energy and adds
// -2 S'(u) e to f. With t = max(u - rs2, 0)/(rc2 - rs2) and d = 1 - t:
// S = d^2 (1 + 2t) and -2 S' = 12 t d / (rc2 - rs2).
template <typename Real, bool kSwitchCoulomb>
__device__ inline Real pair_force(Real u, Real c12, Real c6, Real qq, const Consts<Real>& k,
                                  Real& e) {
  Real rinv = rsqrt_r(u);
  Real r2 = rinv * rinv;
  Real r6 = r2 * r2 * r2;
  Real A = c12 * r6 * r6;
  Real B = c6 * r6;
  Real elj = A - B;
  Real flj = Real(12) * A - Real(6) * B;
  Real ec = qq * rinv;
  Real xs = u - k.rs2;
  xs = xs > Real(0) ? xs : Real(0);
  Real t = xs * k.inv_sw;
  Real d = Real(1) - t;
  Real S = d * d * (Real(1) + Real(2) * t);
  Real g = t * d * k.sw12;
  if (kSwitchCoulomb) {
    Real et = elj + ec;
    e = S * et;
    return S * (flj + ec) * r2 + g * et;
  } else {
    e = S * elj + ec;
    return (S * flj + ec) * r2 + g * elj;
  }
}

struct TaskGeom {
  int64_t cellA, cellB;
  int k;
  int shA[3], shB[3];   // 1 where L is subtracted from that side's coordinate
};

__device__ inline TaskGeom task_geom(int64_t t, int nx, int ny, int nz) {
  TaskGeom g;
  g.cellA = t / kTasksPerCell;
  g.k = (int)(t % kTasksPerCell);
  int ax = (int)(g.cellA % nx);
  int ay = (int)((g.cellA / nx) % ny);
  int az = (int)(g.cellA / ((int64_t)nx * ny));
  int b[3] = {ax + c_off[g.k][0], ay + c_off[g.k][1], az + c_off[g.k][2]};
  int n[3] = {nx, ny, nz};
  for (int d = 0; d < 3; ++d) {
    g.shA[d] = 0;
    g.shB[d] = 0;
    if (b[d] >= n[d]) {      // A is in the last cell: its image moves down by L
      b[d] -= n[d];
      g.shA[d] = 1;
    } else if (b[d] < 0) {   // B is in the last cell: its image moves down by L
      b[d] += n[d];
      g.shB[d] = 1;
    }
  }
  g.cellB = ((int64_t)b[2] * ny + b[1]) * nx + b[0];
  return g;
}

// The dispatcher places workgroup b on XCD b % 8; give each XCD a contiguous range of
// tasks (neighbouring cells) so that its L2 holds their atoms.
__device__ inline int64_t xcd_task(int64_t b, int64_t n_tasks) {
  int64_t per = (n_tasks + 7) / 8;
  return (b % 8) * per + b / 8;
}

template <typename Real>
__device__ inline void block_reduce_energy(double e, double* sE, double* out) {
  sE[threadIdx.x] = e;
  __syncthreads();
  for (int off = kPairThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sE[threadIdx.x] += sE[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sE[0];
}

// Writes (or, when the task spans several tiles, adds) one partial force.
template <typename Real>
__device__ inline void put_partial(const SysArgs<Real>& a, int slot, int c, int64_t s, Real v,
                                   bool accumulate) {
  if (a.flags & MD_ACCUM_F32_ATOMIC) {
    atomicAdd(&a.facc[(int64_t)c * a.n + s], (float)v);
    return;
  }
  Real* p = &a.part[((int64_t)slot * 3 + c) * a.n + s];
  *p = accumulate ? *p + v : v;
}

// ------------------------------------------------------------ predicated ----

template <typename Real, bool kSwitchCoulomb>
__global__ __launch_bounds__(kPairThreads) void k_pair_predicated(SysArgs<Real> a) {
  extern __shared__ unsigned char s_dyn[];
  Real* sLJ = reinterpret_cast<Real*>(s_dyn);
  __shared__ P4<Real> sA[kTile], sB[kTile];
  __shared__ int sTA[kTile], sTB[kTile];
  __shared__ Real sAccJ[kPairThreads / 64][3][kTile];
  __shared__ int sCntJ[kTile];
  __shared__ double sE[kPairThreads];
  __shared__ unsigned long long sDiag[2];

  int64_t t = xcd_task(blockIdx.x, a.n_tasks);
  if (t >= a.n_tasks) return;
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const bool diag = (a.flags & MD_DIAG_COUNTERS) != 0;
  const int nt = a.n_types;
  for (int e = tid; e < 2 * nt * nt; e += kPairThreads) sLJ[e] = a.lj[e];
  if (tid < 2) sDiag[tid] = 0;

  TaskGeom g = task_geom(t, a.nx, a.ny, a.nz);
  const bool self = g.k == 0;
  const int64_t sA0 = a.start[g.cellA], nA = a.start[g.cellA + 1] - sA0;
  const int64_t sB0 = a.start[g.cellB], nB = a.start[g.cellB + 1] - sB0;
  const int slotA = g.k, slotB = self ? 0 : 13 + g.k;
  const bool multi = nA > kTile || nB > kTile;
  Consts<Real> K{a.rc2, a.rs2, a.inv_sw, Real(12) * a.inv_sw};
  Real shA[3], shB[3];
  for (int d = 0; d < 3; ++d) {
    shA[d] = g.shA[d] ? a.L[d] : Real(0);
    shB[d] = g.shB[d] ? a.L[d] : Real(0);
  }

  if (multi && !(a.flags & MD_ACCUM_F32_ATOMIC)) {
    for (int64_t e = tid; e < nA; e += kPairThreads)
      for (int c = 0; c < 3; ++c) a.part[((int64_t)slotA * 3 + c) * a.n + sA0 + e] = Real(0);
    for (int64_t e = tid; e < nB; e += kPairThreads)
      for (int c = 0; c < 3; ++c) a.part[((int64_t)slotB * 3 + c) * a.n + sB0 + e] = Real(0);
  }
  __syncthreads();

  double e_acc = 0.0;
  for (int64_t a0 = 0; a0 < nA; a0 += kTile) {
    const int mA = (int)min<int64_t>(kTile, nA - a0);
    for (int64_t b0 = self ? a0 : 0; b0 < nB; b0 += kTile) {
      const int mB = (int)min<int64_t>(kTile, nB - b0);
      const bool sblock = self && a0 == b0;
      if (tid < mA) {
        P4<Real> p = a.pos[sA0 + a0 + tid];
        p.x -= shA[0];
        p.y -= shA[1];
        p.z -= shA[2];
        p.w *= a.coulomb_k;
        sA[tid] = p;
        sTA[tid] = a.type[sA0 + a0 + tid] * nt;
      }
      if (tid < mB) {
        P4<Real> p = a.pos[sB0 + b0 + tid];
        p.x -= shB[0];
        p.y -= shB[1];
        p.z -= shB[2];
        sB[tid] = p;
        sTB[tid] = a.type[sB0 + b0 + tid];
        sCntJ[tid] = 0;
      }
      for (int e = tid; e < (kPairThreads / 64) * 3 * kTile; e += kPairThreads)
        (&sAccJ[0][0][0])[e] = Real(0);
      __syncthreads();

      Real Fx = 0, Fy = 0, Fz = 0;
      int cnt = 0;
      if (tid < mA) {
        const P4<Real> pi = sA[tid];
        const int ti = sTA[tid];
        // Candidates of this lane: the whole neighbour tile, starting at a lane-dependent
        // position so that the lanes of a wave touch distinct neighbours; on the home
        // tile, the offsets 1..(m-1)/2 (and m/2 for the first half when m is even)
        // cover every unordered pair once.
        int steps, j;
        if (sblock) {
          steps = (mA - 1) / 2 + ((mA % 2 == 0 && tid < mA / 2) ? 1 : 0);
          j = tid;
        } else {
          steps = mB;
          j = tid % mB;
        }
        for (int s = 0; s < steps; ++s) {
          if (sblock) {
            ++j;
            if (j == mA) j = 0;
          }
          const P4<Real> pj = sB[j];
          const Real dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
          const Real u = dist2(dx, dy, dz);
          if (u < K.rc2) {
            const int e2 = 2 * (ti + sTB[j]);
            Real e;
            const Real f = pair_force<Real, kSwitchCoulomb>(u, sLJ[e2], sLJ[e2 + 1],
                                                            pi.w * pj.w, K, e);
            Fx += f * dx;
            Fy += f * dy;
            Fz += f * dz;
            atomicAdd(&sAccJ[wave][0][j], -f * dx);
            atomicAdd(&sAccJ[wave][1][j], -f * dy);
            atomicAdd(&sAccJ[wave][2][j], -f * dz);
            e_acc += (double)e;
            ++cnt;
            if (diag) atomicAdd(&sCntJ[j], 1);
          }
          if (!sblock) {
            ++j;
            if (j == mB) j = 0;
          }
        }
      }
      if (diag && tid == 0) {
        unsigned long long cand = sblock ? (unsigned long long)mA * (mA - 1) / 2
                                         : (unsigned long long)mA * mB;
        atomicAdd(&sDiag[0], cand);
      }
      __syncthreads();
      const bool acc = multi;
      if (tid < mA) {
        Real v[3] = {Fx, Fy, Fz};
        for (int c = 0; c < 3; ++c) {
          if (sblock)
            for (int w = 0; w < kPairThreads / 64; ++w) v[c] += sAccJ[w][c][tid];
          put_partial(a, slotA, c, sA0 + a0 + tid, v[c], acc);
        }
        if (diag) {
          int ci = cnt + (sblock ? sCntJ[tid] : 0);
          atomicAdd(&a.paircount[a.n + sA0 + a0 + tid], ci);
          atomicAdd(&sDiag[1], (unsigned long long)cnt);
        }
      }
      if (!sblock && tid < mB) {
        for (int c = 0; c < 3; ++c) {
          Real v = Real(0);
          for (int w = 0; w < kPairThreads / 64; ++w) v += sAccJ[w][c][tid];
          put_partial(a, slotB, c, sB0 + b0 + tid, v, acc);
        }
        if (diag) atomicAdd(&a.paircount[a.n + sB0 + b0 + tid], sCntJ[tid]);
      }
      __syncthreads();
    }
  }
  // tasks whose A or B cell is empty still own their slots: write zeros
  if (nA == 0 || nB == 0) {
    if (!(a.flags & MD_ACCUM_F32_ATOMIC)) {
      for (int64_t e = tid; e < nA; e += kPairThreads)
        for (int c = 0; c < 3; ++c) a.part[((int64_t)slotA * 3 + c) * a.n + sA0 + e] = Real(0);
      for (int64_t e = tid; e < nB; e += kPairThreads)
        for (int c = 0; c < 3; ++c) a.part[((int64_t)slotB * 3 + c) * a.n + sB0 + e] = Real(0);
    }
  }
  block_reduce_energy<Real>(e_acc, sE, &a.epart[t]);
  if (diag && tid == 0) {
    atomicAdd(&a.hdr->diag[0], sDiag[0]);
    atomicAdd(&a.hdr->diag[1], sDiag[1]);
    atomicAdd(&a.hdr->diag[2], sDiag[1]);
    atomicAdd(&a.hdr->diag[3], sDiag[0]);
    atomicAdd(&a.hdr->diag[4], sDiag[0]);   // every candidate goes through the force arithmetic
  }
}

}  // namespace

template <typename Real>
hipError_t launch_pair(const SysArgs<Real>& a, hipStream_t stream) {
  if (a.n == 0) return hipSuccess;
  if (a.compact) return launch_pair_fs<Real>(a, stream);
  const int64_t blocks = 8 * ((a.n_tasks + 7) / 8);
  const size_t shmem = sizeof(Real) * 2 * a.n_types * a.n_types;
  const bool swc = !(a.flags & MD_COULOMB_TRUNCATED);
  if (swc)
    hipLaunchKernelGGL((k_pair_predicated<Real, true>), dim3((unsigned)blocks),
                       dim3(kPairThreads), shmem, stream, a);
  else
    hipLaunchKernelGGL((k_pair_predicated<Real, false>), dim3((unsigned)blocks),
                       dim3(kPairThreads), shmem, stream, a);
  return hipGetLastError();
}

template hipError_t launch_pair<float>(const SysArgs<float>&, hipStream_t);
template hipError_t launch_pair<double>(const SysArgs<double>&, hipStream_t);

}  // namespace md
