// Compacted pair kernel, full shell: the loop order of Algorithm 1 (Section 2.1)
// -- foreach home cell, foreach of its 27 neighbour cells, foreach home atom,
// foreach neighbour atom, test the cutoff and accumulate the force on the home atom --
// with the dynamic data flow of the enhanced design (Section 4.2, Fig. 4, Algorithm 3):
// many cutoff filters feed one force stage through FIFOs, and the force stage only
// ever works on pairs that passed.
//
// One workgroup (8 waves) takes half of the atoms of one home cell. It stages the
// atoms of the 27 neighbour cell images in LDS (periodic images shifted exactly:
// the side lying in the last cell of an axis subtracts L, Sterbenz-exact), then each
// wave takes groups of 8 home atoms:
//   filter  -- for every 64 neighbour atoms (one per lane) and each of the 8 home
//              atoms: the squared distance, the strict test u < rc^2, a wave ballot,
//              and a prefix count (mbcnt) that appends the passing neighbour indices
//              to that home atom's FIFO in LDS (8 "distance PEs" per wave);
//   force   -- whenever a FIFO holds 64 entries, one dense pass over them with every
//              lane busy (the "force PE"), summing the force on the home atom in
//              registers.
// Each home atom is owned by one wave, so no atomics are needed and every sum runs in
// a fixed order. At the end the 64 lane partials are added per 16-lane row in a
// fixed DPP order and the four row sums in 64-bit fixed point (2^-32 kcal/mol/A),
// exactly. Every pair is evaluated from both of its atoms, as in Algorithm 1.
#include "md_common.hpp"

namespace md {
namespace {

constexpr int kNW = 16;             // waves per workgroup
constexpr int kThreads = 64 * kNW;
constexpr int kQ = 4;               // home atoms filtered together by one wave, one FIFO each
constexpr int kDrain = 2;           // force batches of 64 drained together from a full FIFO
constexpr int kFifo = 64 * (kDrain + 1);  // FIFO entries: (neighbour type << 16) | index
constexpr int kSplit = kFsSplit;    // workgroups per home cell
constexpr int kLdsBytes = 160 * 1024;
constexpr float kMargin = 0.05f;    // A^2 added to rc^2 by the expanded-form prefilter
constexpr float kFar = 1.0e18f;     // |coordinate| that fails every cutoff test; absent home
                                    // atoms use +kFar, absent neighbours -kFar

// The 27 neighbour images, the home cell first.
__constant__ int8_t c_img[27][3] = {
    {0, 0, 0},    {-1, -1, -1}, {0, -1, -1}, {1, -1, -1}, {-1, 0, -1}, {0, 0, -1}, {1, 0, -1},
    {-1, 1, -1},  {0, 1, -1},   {1, 1, -1},  {-1, -1, 0}, {0, -1, 0},  {1, -1, 0}, {-1, 0, 0},
    {1, 0, 0},    {-1, 1, 0},   {0, 1, 0},   {1, 1, 0},   {-1, -1, 1}, {0, -1, 1}, {1, -1, 1},
    {-1, 0, 1},   {0, 0, 1},    {1, 0, 1},   {-1, 1, 1},  {0, 1, 1},   {1, 1, 1}};

struct Img {
  int start;   // first sorted index of the cell
  int count;
  int off;     // position in the neighbour list
  int grp;     // bit d: image lies at +L along d (the home side subtracts L)
  int jsh;     // bit d: image lies at -L along d (the neighbour side subtracts L)
};

struct StaticLds {
  uint32_t fifo[kNW][kQ * kFifo + 64];  // per home atom: passing neighbours; last 64: lanes
                                        // that did not pass write here (never read)
  Img img[27];
  int grp_begin[9];                 // neighbour-list position where group g starts
  int next;                         // next group of home atoms to hand out
};

__device__ inline float rowsum16(float v) {
  // fixed butterfly: xor 1, xor 2, mirror within 8, mirror within 16
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0xB1, 0xf, 0xf, false));
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x4E, 0xf, 0xf, false));
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x141, 0xf, 0xf, false));
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x140, 0xf, 0xf, false));
  return v;
}

// float -> 64-bit fixed point, one unit = 2^-32, round to nearest even, exact.
__device__ inline long long to_fixed(float v, uint32_t& st) {
  float a = fabsf(v);
  if (!(a < 2147483648.0f)) {
    st |= MD_STATUS_FIXED_OVERFLOW;
    return 0;
  }
  float hi = floorf(a);
  float fr = a - hi;                                // exact
  float lo = rintf(fr * 4294967296.0f);             // exact scaling; < 2^32
  unsigned long long m =
      ((unsigned long long)(unsigned)hi << 32) + (unsigned long long)(unsigned)lo;
  return v < 0.f ? -(long long)m : (long long)m;
}

__device__ inline long long readlane64(long long v, int lane) {
  unsigned lo = __builtin_amdgcn_readlane((int)(unsigned)(v & 0xffffffffull), lane);
  unsigned hi = __builtin_amdgcn_readlane((int)(unsigned)((unsigned long long)v >> 32), lane);
  return (long long)(((unsigned long long)hi << 32) | lo);
}

// Scalar pair force and energy; identical arithmetic to the half-shell kernels.
template <bool kSwitchCoulomb>
__device__ inline float pair_f(float u, float c12, float c6, float qq, float rs2, float inv_sw,
                               float sw12, float& e) {
  float rinv = __builtin_amdgcn_rsqf(u);
  float r2 = rinv * rinv;
  float r6 = r2 * r2 * r2;
  float A = c12 * r6 * r6;
  float B = c6 * r6;
  float elj = A - B;
  float flj = 12.f * A - 6.f * B;
  float ec = qq * rinv;
  float xs = fmaxf(u - rs2, 0.f);
  float t = xs * inv_sw;
  float d = 1.f - t;
  float S = d * d * (1.f + 2.f * t);
  float g = t * d * sw12;
  if (kSwitchCoulomb) {
    float et = elj + ec;
    e = S * et;
    return S * (flj + ec) * r2 + g * et;
  }
  e = S * elj + ec;
  return (S * flj + ec) * r2 + g * elj;
}

// v = bit `lane` of mask ? a : b, as one v_cndmask on the mask (keeps the compiler from
// turning the select into exec-masked branches)
__device__ inline int select_by_mask(unsigned long long mask, int a, int b) {
  int r;
  __asm__ volatile("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(r) : "v"(b), "v"(a), "s"(mask));
  return r;
}

__device__ inline int64_t xcd_unit(int64_t b, int64_t n_units) {
  int64_t per = (n_units + 7) / 8;
  return (b % 8) * per + b / 8;
}

template <bool kSwitchCoulomb>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4, 4)))
void k_pair_fs(SysArgs<float> a, int cap) {
  // dynamic LDS: neighbour (x,y,z,q) [cap] | neighbour type [cap] | LJ table [2 nt^2]
  extern __shared__ __attribute__((aligned(16))) unsigned char s_dyn[];
  float4* sJ = reinterpret_cast<float4*>(s_dyn);
  uint8_t* sT = s_dyn + 16 * (size_t)cap;
  float* sLJ = reinterpret_cast<float*>(s_dyn + 17 * (size_t)cap);
  __shared__ StaticLds S;

  const int64_t n_units = a.n_cells * kSplit;
  const int64_t unit = xcd_unit(blockIdx.x, n_units);
  if (unit >= n_units) return;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t cellA = unit / kSplit;
  const int half = (int)(unit % kSplit);
  const int nt = a.n_types;
  const bool diag = (a.flags & MD_DIAG_COUNTERS) != 0;
  const bool f32 = (a.flags & MD_ACCUM_F32_ATOMIC) != 0;
  const float rc2 = a.rc2, rs2 = a.rs2, inv_sw = a.inv_sw, sw12 = 12.f * a.inv_sw;
  const float kc = a.coulomb_k;
  const float L0 = a.L[0], L1 = a.L[1], L2 = a.L[2];

  for (int e = tid; e < 2 * nt * nt; e += kThreads) sLJ[e] = a.lj[e];
  const int sA = a.start[cellA];
  const int nA = a.start[cellA + 1] - sA;
  const int ib0 = (int)(((int64_t)half * nA) / kSplit);
  const int ib1 = (int)(((int64_t)(half + 1) * nA) / kSplit);

  // image table: one lane per image (independent loads), then the group order
  if (tid < 27) {
    const int nd[3] = {a.nx, a.ny, a.nz};
    const int ac[3] = {(int)(cellA % a.nx), (int)((cellA / a.nx) % a.ny),
                       (int)(cellA / ((int64_t)a.nx * a.ny))};
    int b[3], grp = 0, jsh = 0;
    for (int d = 0; d < 3; ++d) {
      b[d] = ac[d] + c_img[tid][d];
      if (b[d] >= nd[d]) {
        b[d] -= nd[d];
        grp |= 1 << d;
      } else if (b[d] < 0) {
        b[d] += nd[d];
        jsh |= 1 << d;
      }
    }
    const int64_t cb = ((int64_t)b[2] * a.ny + b[1]) * a.nx + b[0];
    const int st0 = a.start[cb], st1 = a.start[cb + 1];
    S.img[tid].start = st0;
    S.img[tid].count = st1 - st0;
    S.img[tid].grp = grp;
    S.img[tid].jsh = jsh;
    // position in the neighbour list: images ordered by group, then by image index
    // (the home image, group 0, first)
    int off = 0, gb = 0;
    for (int mm = 0; mm < 27; ++mm) {
      const int gm = __builtin_amdgcn_readlane(grp, mm);
      const int cm = __builtin_amdgcn_readlane(st1 - st0, mm);
      off += (gm < grp || (gm == grp && mm < tid)) ? cm : 0;
      gb += (tid < 9 && gm < tid) ? cm : 0;      // lane g < 9: start of group g
    }
    S.img[tid].off = off;
    if (tid < 9) S.grp_begin[tid] = gb;
  }
  __syncthreads();

  const int total = S.grp_begin[8];
  const int n_grp_q = (ib1 - ib0 + kQ - 1) / kQ;
  double e_wave = 0.0;
  unsigned long long pass_count = 0;
  uint32_t st = 0;
  uint32_t* fifo = &S.fifo[w][0];

  for (int P0 = 0; P0 < total; P0 += cap) {
    const int P1 = min(total, P0 + cap);
    // stage the neighbour-list slice [P0, P1): wave w copies images w and w + 16, issuing
    // all loads of an image (up to 4 x 64 atoms per round) before its LDS stores
    for (int m = w; m < 27; m += kNW) {
      const Img im = S.img[m];
      const int lo = max(im.off, P0), hi = min(im.off + im.count, P1);
      for (int e0 = lo; e0 < hi; e0 += 4 * 64) {
        P4<float> v[4];
        int tv[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int e = e0 + 64 * r + lane;
          const int src = im.start + (min(e, hi - 1) - im.off);
          v[r] = a.pos[src];
          tv[r] = a.type[src];
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int e = e0 + 64 * r + lane;
          if (e < hi) {
            const float x = (im.jsh & 1) ? v[r].x - L0 : v[r].x;
            const float y = (im.jsh & 2) ? v[r].y - L1 : v[r].y;
            const float z = (im.jsh & 4) ? v[r].z - L2 : v[r].z;
            sJ[e - P0] = make_float4(x, y, z, v[r].w);
            sT[e - P0] = (uint8_t)tv[r];
          }
        }
      }
    }
    if (tid == 0) S.next = 0;
    __syncthreads();

    while (true) {
      int o = 0;
      if (lane == 0) o = atomicAdd(&S.next, 1);
      o = __builtin_amdgcn_readfirstlane(__shfl(o, 0));
      if (o >= n_grp_q) break;
      const int ib = ib0 + kQ * o;

      float xi[kQ], yi[kQ], zi[kQ], kq[kQ], fx[kQ], fy[kQ], fz[kQ];
      int ti[kQ], tl[kQ];
      unsigned cnt[kQ];
#pragma unroll
      for (int k = 0; k < kQ; ++k) {
        const bool v = ib + k < ib1;
        const int s = sA + (v ? ib + k : ib0);
        const P4<float> p = a.pos[s];
        xi[k] = v ? p.x : kFar;   // an absent home atom fails every test
        yi[k] = p.y;
        zi[k] = p.z;
        kq[k] = kc * p.w;
        ti[k] = a.type[s] * nt;
        fx[k] = fy[k] = fz[k] = 0.f;
        tl[k] = 0;
        cnt[k] = 0;
      }
      float e_lane = 0.f;

      for (int g = 0; g < 8; ++g) {
        const int G0 = max(S.grp_begin[g], P0), G1 = min(S.grp_begin[g + 1], P1);
        if (G0 >= G1) continue;
        const int r0 = G0 - P0, r1 = G1 - P0;
        // home coordinates in this group's frame: subtract L where the images lie at +L
        float xs[kQ], ys[kQ], zs[kQ];
        // prefilter terms relative to the origin o (the home cell's first atom, this frame):
        // |x_i - x_j|^2 = c_i + c_j - 2 r_i . r_j with r = x - o, c = |r|^2
        float ax[kQ], ay[kQ], az[kQ], thr[kQ];
        const float ox = xi[0] - ((g & 1) ? L0 : 0.f), oy = yi[0] - ((g & 2) ? L1 : 0.f),
                    oz = zi[0] - ((g & 4) ? L2 : 0.f);
#pragma unroll
        for (int k = 0; k < kQ; ++k) {
          xs[k] = (g & 1) ? xi[k] - L0 : xi[k];
          ys[k] = (g & 2) ? yi[k] - L1 : yi[k];
          zs[k] = (g & 4) ? zi[k] - L2 : zi[k];
          const float rx = xs[k] - ox, ry = ys[k] - oy, rz = zs[k] - oz;
          ax[k] = -2.f * rx;
          ay[k] = -2.f * ry;
          az[k] = -2.f * rz;
          thr[k] = (rc2 + kMargin) - fmaf(rz, rz, fmaf(ry, ry, rx * rx));
        }

        // dense force passes over the first c entries of FIFO k (c <= 64 * kDrain): the exact
        // cutoff test (u < rc^2; u > 0 drops the home atom itself) and the force. All LDS
        // reads of the kDrain batches are issued before any arithmetic.
        auto force = [&](int k, int c) __attribute__((always_inline)) {
          uint32_t ent[kDrain];
          float4 pj[kDrain];
          float c12[kDrain], c6[kDrain];
#pragma unroll
          for (int b = 0; b < kDrain; ++b) ent[b] = fifo[k * kFifo + 64 * b + lane];
#pragma unroll
          for (int b = 0; b < kDrain; ++b) {
            const bool in = 64 * b + lane < c;
            const int jj = in ? (int)(ent[b] & 0xffffu) : r0;
            const int tj = in ? (int)(ent[b] >> 16) : 0;
            pj[b] = sJ[jj];
            const int e2 = 2 * (ti[k] + tj);
            c12[b] = sLJ[e2];
            c6[b] = sLJ[e2 + 1];
          }
#pragma unroll
          for (int b = 0; b < kDrain; ++b) {
            const bool in = 64 * b + lane < c;
            const float dx = xs[k] - pj[b].x, dy = ys[k] - pj[b].y, dz = zs[k] - pj[b].z;
            const float u = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
            const bool lv = in && u < rc2 && u > 0.f;
            float e;
            float f = pair_f<kSwitchCoulomb>(u, c12[b], c6[b], kq[k] * pj[b].w, rs2, inv_sw, sw12, e);
            f = lv ? f : 0.f;
            e = lv ? e : 0.f;
            fx[k] = fmaf(f, dx, fx[k]);
            fy[k] = fmaf(f, dy, fy[k]);
            fz[k] = fmaf(f, dz, fz[k]);
            e_lane += e;
            cnt[k] += __builtin_popcountll(__builtin_amdgcn_ballot_w64(lv));
          }
          // drop the first c entries; the remainder (fewer than 64) moves to the front
          const int rem = tl[k] - c;
          if (rem > 0) {
            uint32_t v = 0;
            if (lane < rem) v = fifo[k * kFifo + c + lane];
            if (lane < rem) fifo[k * kFifo + lane] = v;
          }
          tl[k] = rem;
        };

        // software pipeline: the next batch's neighbour is loaded one batch ahead
        int jr = min(r0 + lane, r1 - 1);
        float4 pn = sJ[jr];
        uint32_t cn = ((uint32_t)sT[jr] << 16) | (uint32_t)jr;
        for (int jb = r0; jb < r1; jb += 64) {
          const int jv = jb + lane;
          const bool last = jb + 64 >= r1;
          float4 pj = pn;
          const uint32_t code = cn;
          if (!last) {
            const int jn = min(jv + 64, r1 - 1);
            pn = sJ[jn];
            cn = ((uint32_t)sT[jn] << 16) | (uint32_t)jn;
          }
          if (last) pj.x = jv < r1 ? pj.x : -kFar;   // opposite sign to the absent-home sentinel
          const float rx = pj.x - ox, ry = pj.y - oy, rz = pj.z - oz;
          const float cj = fmaf(rz, rz, fmaf(ry, ry, rx * rx));
          float t[kQ];
#pragma unroll
          for (int k = 0; k < kQ; ++k) t[k] = fmaf(ax[k], rx, cj);
#pragma unroll
          for (int k = 0; k < kQ; ++k) t[k] = fmaf(ay[k], ry, t[k]);
#pragma unroll
          for (int k = 0; k < kQ; ++k) t[k] = fmaf(az[k], rz, t[k]);
          unsigned long long m[kQ];
#pragma unroll
          for (int k = 0; k < kQ; ++k) m[k] = __builtin_amdgcn_ballot_w64(t[k] < thr[k]);
          // every lane writes: passing lanes to their FIFO slot, the others to their own
          // dump slot, so no exec-mask changes are needed
          int idx[kQ];
#pragma unroll
          for (int k = 0; k < kQ; ++k) {
            const int rank = (int)__builtin_amdgcn_mbcnt_hi(
                (unsigned)(m[k] >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m[k], 0u));
            idx[k] = select_by_mask(m[k], k * kFifo + tl[k] + rank, kQ * kFifo + lane);
          }
#pragma unroll
          for (int k = 0; k < kQ; ++k) fifo[idx[k]] = code;
#pragma unroll
          for (int k = 0; k < kQ; ++k) tl[k] += __builtin_popcountll(m[k]);
          // drain full FIFOs (kDrain batches at a time); on the group's last batch drain
          // everything (the home side changes frame in the next group)
          const int thr_n = last ? 1 : 64 * kDrain;
#pragma unroll
          for (int k = 0; k < kQ; ++k) {
            while (tl[k] >= thr_n) force(k, tl[k] < 64 * kDrain ? tl[k] : 64 * kDrain);
          }
        }
      }

      // per home atom: fixed-order row sums, then the four rows in 64-bit fixed point
#pragma unroll
      for (int k = 0; k < kQ; ++k) {
        if (ib + k >= ib1) continue;
        const int64_t s = sA + ib + k;
        const float comp[3] = {fx[k], fy[k], fz[k]};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const float r = rowsum16(comp[c]);
          if (f32) {
            const float r0 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, r), 0));
            const float r1 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, r), 16));
            const float r2 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, r), 32));
            const float r3 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, r), 48));
            const float tot = (r0 + r1) + (r2 + r3);
            if (lane == 0) {
              float* dst = &a.facc[(int64_t)c * a.n + s];
              *dst = P0 == 0 ? tot : *dst + tot;
            }
          } else {
            const long long q = to_fixed(r, st);
            const long long tot = readlane64(q, 0) + readlane64(q, 16) + readlane64(q, 32) +
                                  readlane64(q, 48);
            if (lane == 0) {
              long long* dst = &a.acc64[(int64_t)c * a.n + s];
              *dst = P0 == 0 ? tot : *dst + tot;
            }
          }
        }
        if (diag && lane == 0) {
          int* dst = &a.paircount[a.n + s];
          *dst = P0 == 0 ? (int)cnt[k] : *dst + (int)cnt[k];
        }
        pass_count += cnt[k];
      }
      e_wave += (double)e_lane;
    }
    __syncthreads();
  }

  // workgroup energy: each pair was seen from both atoms
  double* sE = reinterpret_cast<double*>(s_dyn);
  sE[tid] = e_wave;
  __syncthreads();
  for (int off = kThreads / 2; off > 0; off >>= 1) {
    if (tid < off) sE[tid] += sE[tid + off];
    __syncthreads();
  }
  if (tid == 0) a.epart[unit] = 0.5 * sE[0];
  if (st) atomicOr(&a.hdr->status, st);
  if (diag && lane == 0) {
    // candidates: every (home atom, other neighbour-list atom), counted from both atoms
    if (w == 0) {
      const unsigned long long cand =
          (unsigned long long)(ib1 - ib0) * (unsigned long long)(total - 1);
      atomicAdd(&a.hdr->diag[0], cand);
    }
    atomicAdd(&a.hdr->diag[1], pass_count);
    atomicAdd(&a.hdr->diag[2], pass_count);
  }
}

}  // namespace

// Neighbour atoms staged in LDS per pass for n_types types (a multiple of 64).
static int fs_cap(int n_types) {
  const int avail = kLdsBytes - (int)sizeof(StaticLds) - (int)sizeof(float) * 2 * n_types * n_types;
  int cap = avail / 17;
  cap -= cap % 64;
  return cap;
}

size_t pair_fs_lds_bytes(int n_types) {
  return (size_t)17 * fs_cap(n_types) + sizeof(float) * 2 * n_types * n_types;
}

hipError_t launch_pair_fs(const SysArgs<float>& a, hipStream_t stream) {
  if (a.n == 0) return hipSuccess;
  const int64_t units = a.n_cells * kSplit;
  const int64_t blocks = 8 * ((units + 7) / 8);
  const int cap = fs_cap(a.n_types);
  const size_t shmem = pair_fs_lds_bytes(a.n_types);
  if (!(a.flags & MD_COULOMB_TRUNCATED))
    hipLaunchKernelGGL(k_pair_fs<true>, dim3((unsigned)blocks), dim3(kThreads), shmem, stream, a,
                       cap);
  else
    hipLaunchKernelGGL(k_pair_fs<false>, dim3((unsigned)blocks), dim3(kThreads), shmem, stream, a,
                       cap);
  return hipGetLastError();
}

}  // namespace md
