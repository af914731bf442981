// Compacted pair kernel: the loop order of Algorithm 1 (Section 2.1) -- foreach home
// cell, foreach of its neighbour cells, foreach home atom, foreach neighbour atom, test
// the cutoff and accumulate the force -- with the dynamic data flow of the enhanced
// design (Section 5.2, Fig. 4; Algorithm 3): several cutoff filters feed one force stage
// through FIFOs, and the force stage only ever works on pairs that passed.
//
// One workgroup (16 waves) takes one home cell. It stages the atoms of its neighbour-
// cell images in LDS, periodic images shifted exactly (the side lying in the
// last cell of an axis subtracts L, which is Sterbenz-exact). Each z half of a cell is
// sorted by x, so one z half of the images of one (dy, dz) row, laid out in x order,
// forms one x-sorted "segment".
// Each wave takes groups of kQ home atoms (consecutive in x) and, per segment, only the
// slice whose x lies within r_cut of the group, found by a binary search (one lane
// per segment):
//   filter  -- for every 64 neighbour atoms (one per lane) and each of the kQ home
//              atoms: a conservative expanded-form distance test (three FMAs against a
//              precomputed |r_j - o|^2), a wave ballot, and a prefix count (mbcnt) that
//              appends the passing neighbour index to that home atom's FIFO in LDS
//              (kQ "distance PEs" per wave);
//   force   -- whenever a FIFO holds kDrain x 64 entries, dense passes over them with
//              every lane busy (the "force PE"): the exact distance, the strict test
//              u < rc^2, and the force summed on the home atom in registers.
// Each home atom is owned by one wave and its sum runs in a fixed order: the 64 lane
// partials are added in one fixed order (wave halves and rows exchanging partial sums,
// then a butterfly within a row) and the total converted to 64-bit fixed point
// (2^-28 kcal/mol/A, one rounding); lane energies are summed in 64-bit fixed point (2^-24 kcal/mol),
// so the energy does not depend on how groups of home atoms were spread over the waves
// either.
//
// Two shells:
//   full (kHalf = false) -- every pair is evaluated from both of its atoms, as in
//              Algorithm 1, over the 27 images; each atom's sum is written by the one
//              wave that owns it, so no atomics are needed;
//   half (kHalf = true)  -- every pair is evaluated once (Newton's third law, F_j = -F_i):
//              the home cell with j > i and the 13 images ahead of it. The force on the
//              neighbour atom, -f dx rounded once to a multiple of 2^-24 (through one float64
//              fused multiply-add), is added in 64-bit fixed
//              point into an LDS accumulator per staged atom (integer atomics, so the sum
//              does not depend on the order of the adds), and the accumulators go to the
//              per-atom sums with 64-bit global integer atomics when the workgroup is
//              done. Integer addition is associative: the same bits on every run.
//
// Two precisions, one template (Real):
//   float  -- the hot path. The staged c_j carries the atom type in its low mantissa bits;
//             the neighbour-side force is rounded to 2^-24 units in one 64-bit integer.
//   double -- float64 throughout: the same staging, segments, windows, filter, FIFOs and
//             force passes, with the squared distance rounded term by term as a plain
//             float64 evaluation of dx^2 + dy^2 + dz^2 (so the cutoff decides like the
//             definition). Per-atom sums and energies use a two-word fixed point,
//             v = hi 2^-20 + lo 2^-72 (both int64), exact for every float64 partial above
//             2^-20 kcal/mol/A, so they too are the same bits on every run; types live in
//             an LDS array of their own.
#include <type_traits>

#include "md_common.hpp"

namespace md {
namespace {

constexpr int kNW = 16;             // waves per workgroup
constexpr int kThreads = 64 * kNW;
constexpr int kQ = 4;               // home atoms filtered together by one wave, one FIFO each
static_assert(kQ % 4 == 0, "FIFO appends are written four home atoms at a time");
static_assert(kNW % 4 == 0 && kNW * 64 <= 1024, "waves per workgroup");
// Force batches of 64 drained together from a full FIFO (kDrain, a template parameter of
// the kernel: 2 by default, 1 to 4 for the drain-depth sweep); a FIFO holds
// 64 (kDrain + 1) uint16 neighbour indices.
constexpr int kDrainDefault = 2;
__host__ __device__ constexpr int fifo_entries(int drain) { return 64 * (drain + 1); }
constexpr int kMaxSeg = 36;         // 9 (dy, dz) rows x 2 z halves, each split at most once by
                                    // an x wrap
constexpr int kLdsBytes = 160 * 1024;
constexpr float kWin = 1.0e-3f;     // A added to r_cut for the x-window
constexpr float kBigU = 1.0e30f;    // squared distance given to lanes that must add nothing
// Range of the per-atom 64-bit fixed-point sums of the float32 path: units of 2^-28
// kcal/mol/A, magnitudes below 2^35. In the half shell an atom's sum gathers one
// neighbour-side partial from each of the 14 images that stage it, in each of the n_split
// workgroups of the staging cell (its home image and the 13 cells that have its cell
// ahead), each below 2^27 (kNbrPartialMax, also the bound of one pair's term), and one
// home-side partial per LDS slice of its home cell's neighbour list, S of them, sharing
// what is left: (2^35 - 14 n_split 2^27) / S each. In the full shell an atom's S home-side
// partials are each below 2^35 / S. Every partial is checked, so a sum can never wrap.
constexpr float kNbrPartialMax = 134217728.f;      // 2^27
constexpr float kAccRange = 34359738368.f;         // 2^35
static_assert(kMaxTypes <= 64, "a type must fit the low 6 bits of a staged c_j");

// Staged atom (x, y, z, c_j) and LJ (c12, c6) vector types of each precision.
template <typename Real>
using V4 = std::conditional_t<sizeof(Real) == 4, float4, double4>;
template <typename Real>
using V2 = std::conditional_t<sizeof(Real) == 4, float2, double2>;
// 64-bit words per component of a per-atom fixed-point sum: 1 (float), 2 (double: hi, lo)
template <typename Real>
constexpr int kAccWords = sizeof(Real) == 8 ? 2 : 1;

__device__ inline float mad(float a, float b, float c) { return fmaf(a, b, c); }
__device__ inline double mad(double a, double b, double c) { return fma(a, b, c); }
__device__ inline float vmin(float a, float b) { return fminf(a, b); }
__device__ inline double vmin(double a, double b) { return fmin(a, b); }
__device__ inline float vmax(float a, float b) { return fmaxf(a, b); }
__device__ inline double vmax(double a, double b) { return fmax(a, b); }
__device__ inline float vsqrt(float a) { return __builtin_sqrtf(a); }
__device__ inline double vsqrt(double a) { return sqrt(a); }
// square root of the x-window's half-width: float32's hardware square root (within 1 ulp,
// far inside the window's 1e-3 A margin), float64's correctly rounded one
__device__ inline float wsqrt(float a) { return __builtin_amdgcn_sqrtf(a); }
__device__ inline double wsqrt(double a) { return sqrt(a); }
__device__ inline float4 mk4(float x, float y, float z, float w) { return make_float4(x, y, z, w); }
__device__ inline double4 mk4(double x, double y, double z, double w) {
  return make_double4(x, y, z, w);
}
template <typename Real>
__device__ inline V2<Real> mk2(Real x, Real y) {
  if constexpr (sizeof(Real) == 4) return make_float2(x, y); else return make_double2(x, y);
}

// Squared distance. float: fused, as the filter's test. double: each product and sum
// rounded on its own, in the order ((dx^2 + dy^2) + dz^2) of a plain float64 evaluation.
__device__ inline float dist2(float dx, float dy, float dz) {
  return fmaf(dz, dz, fmaf(dy, dy, dx * dx));
}
__device__ inline double dist2(double dx, double dy, double dz) {
  return __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
}

// The 27 neighbour images.
__constant__ int8_t c_img[27][3] = {
    {0, 0, 0},    {-1, -1, -1}, {0, -1, -1}, {1, -1, -1}, {-1, 0, -1}, {0, 0, -1}, {1, 0, -1},
    {-1, 1, -1},  {0, 1, -1},   {1, 1, -1},  {-1, -1, 0}, {0, -1, 0},  {1, -1, 0}, {-1, 0, 0},
    {1, 0, 0},    {-1, 1, 0},   {0, 1, 0},   {1, 1, 0},   {-1, -1, 1}, {0, -1, 1}, {1, -1, 1},
    {-1, 0, 1},   {0, 0, 1},    {1, 0, 1},   {-1, 1, 1},  {0, 1, 1},   {1, 1, 1}};

// Half shell: the home image and the 13 images ahead of it (dz = +1; dz = 0 and
// dy = +1; dz = dy = 0 and dx = +1). Of two opposite offsets exactly one is here, so
// every pair of distinct images is visited once, from the cell that has the other ahead.
__constant__ int8_t c_himg[14][3] = {
    {0, 0, 0},  {-1, -1, 1}, {0, -1, 1}, {1, -1, 1}, {-1, 0, 1}, {0, 0, 1}, {1, 0, 1},
    {-1, 1, 1}, {0, 1, 1},   {1, 1, 1},  {-1, 1, 0}, {0, 1, 0},  {1, 1, 0}, {1, 0, 0}};

struct Img {
  int start;   // first sorted index of the cell
  int count;
  int n0;      // atoms in the cell's lower z half (they come first)
  int off[2];  // neighbour-list position of the lower and upper halves
  int grp;     // bit d: image lies at +L along d (the home side subtracts L)
  int jsh;     // bit d: image lies at -L along d (the neighbour side subtracts L)
};

// A segment: one z half of the images of one (dy, dz) row with one shift class, in x
// order. Its slab bounds y0..y1, z0..z1 are in the home cell's frame.
struct alignas(16) Seg {
  float y0, y1, z0, z1;   // first: one 16-byte load
  int begin, end;         // neighbour-list positions
  int grp;
};

// Workgroup header in LDS.
struct Hdr {
  Img img[27];
  Seg seg[kMaxSeg];
  int n_seg;
  int total;        // neighbour-list length
  int iters;        // binary-search steps that cover the longest segment
  int next;         // next group of home atoms to hand out
  int done;         // waves that have added their energy to esum
  long long esum[2];   // the workgroup's energy (float64: high and low words)
};

// LDS layout in bytes: header | FIFOs | LJ (c12, c6) [nt^2] | (x, y, z, |r - o_g|^2, in
// float32 with the type in its low bits) [cap] | q [cap] | (float64) type [cap], and for
// the half shell the neighbour-side accumulators (x, y, z) x kAccWords int64 [cap] and,
// with counters, partner counts int32 [cap]
struct Lds {
  int hdr, fifo, lj, f4, q, typ, jacc, jcnt, total;
};

__host__ __device__ constexpr int align_up(int v, int a) { return (v + a - 1) / a * a; }

template <typename Real>
__host__ __device__ inline int slot_bytes(bool half, bool diag) {
  constexpr int R = (int)sizeof(Real);
  return 5 * R + (R == 8 ? 4 : 0) + (half ? 24 * kAccWords<Real> + (diag ? 4 : 0) : 0);
}

template <typename Real>
__host__ __device__ inline Lds lds_layout(int cap, int n_types, bool half, bool diag, int drain) {
  constexpr int R = (int)sizeof(Real);
  Lds L;
  L.hdr = 0;
  L.fifo = align_up(L.hdr + (int)sizeof(Hdr), 16);
  L.lj = align_up(L.fifo + 2 * kNW * kQ * fifo_entries(drain), 16);
  L.f4 = align_up(L.lj + 2 * R * n_types * n_types, 4 * R);
  L.q = L.f4 + 4 * R * cap;
  L.typ = L.q + R * cap;
  const int end = L.typ + (R == 8 ? 4 * cap : 0);
  L.jacc = align_up(end, 16);
  L.jcnt = L.jacc + (half ? 24 * kAccWords<Real> * cap : 0);
  L.total = half ? L.jcnt + (diag ? 4 * cap : 0) : end;
  return L;
}

__device__ inline float rowsum16(float v) {
  // fixed butterfly: xor 1, xor 2, mirror within 8, mirror within 16
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0xB1, 0xf, 0xf, false));
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x4E, 0xf, 0xf, false));
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x141, 0xf, 0xf, false));
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x140, 0xf, 0xf, false));
  return v;
}

// Round to nearest even of s to a 64-bit integer, for s a float64 integer or |s| < 2^51:
// below 2^51 the add of 1.5 * 2^52 rounds s once to an integer, which the low bits of the
// sum then hold (as the neighbour side's round_prod_2m24); larger s are integers already
// (a float32 value scaled by a power of two) and take the library conversion.
__device__ inline long long round_to_i64(double s) {
  if (fabs(s) < 2251799813685248.0)   // 2^51
    return __builtin_bit_cast(long long, s + 6755399441055744.0) - 0x4338000000000000ll;
  return __double2ll_rn(s);
}

// float -> 64-bit fixed point, one unit = 2^-28, round to nearest even, exact but for
// that one rounding (v 2^28 is exact in float64).
__device__ inline long long to_fixed(float v, uint32_t& st) {
  if (!(fabsf(v) < kAccRange)) {
    st |= MD_STATUS_FIXED_OVERFLOW;
    return 0;
  }
  return round_to_i64((double)v * 268435456.0);
}

// round(a b 2^24) (to nearest even) as a 64-bit integer, for float32 a, b with
// |a b| < 2^27: the product is exact in float64, and the fused add of 1.5 * 2^28 rounds it
// once to a multiple of 2^-24 (the ulp of values in [2^28, 2^29)), so the bit pattern of
// the sum differs from that of 1.5 * 2^28 by exactly the rounded product in units of 2^-24.
__device__ inline long long round_prod_2m24(double a, float b) {
  const double t = fma(a, (double)b, 402653184.0);
  return __builtin_bit_cast(long long, t) - 0x41b8000000000000ll;
}

// Two-word fixed point of the float64 path: v = hi 2^-20 + lo 2^-72 with hi = round(v 2^20)
// and lo = round((v 2^20 - hi) 2^52), for |v| < 2^31. Both roundings are adds of
// 1.5 * 2^52, as in round_to_i64; v 2^20 - hi is exact (Sterbenz, or hi = 0), so the pair
// holds v exactly whenever |v| >= 2^-20, and to 2^-73 otherwise.
struct Fix2 {
  long long hi, lo;
};
__device__ inline Fix2 to_fix2(double v) {
  const double M = 6755399441055744.0;
  const double s = v * 1048576.0;                       // 2^20, exact
  const double t = s + M;                               // s rounded to an integer
  const double r = (s - (t - M)) * 4503599627370496.0;  // remainder (|r| <= 0.5) times 2^52
  const double t2 = r + M;
  return Fix2{__builtin_bit_cast(long long, t) - 0x4338000000000000ll,
              __builtin_bit_cast(long long, t2) - 0x4338000000000000ll};
}
// hi 2^-20 + lo 2^-72 with lo reduced into [0, 2^52) and its carry moved to hi.
__device__ inline Fix2 normalize2(long long hi, long long lo) {
  return Fix2{hi + (lo >> 52), lo & ((1ll << 52) - 1)};
}
__device__ inline double from_fix2(long long hi, long long lo) {
  return (double)hi * 9.5367431640625e-07 + (double)lo * 2.117582368135751e-22;   // 2^-20, 2^-72
}

__device__ inline void lds_add(long long* p, long long v) {
  __hip_atomic_fetch_add(reinterpret_cast<unsigned long long*>(p), (unsigned long long)v,
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ inline void global_add(long long* p, long long v) {
  __hip_atomic_fetch_add(reinterpret_cast<unsigned long long*>(p), (unsigned long long)v,
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Forms of the Coulomb term (kCoul):
//   kCoulSwitched  the whole pair energy (LJ and Coulomb) is switched;
//   kCoulPlain     only the LJ energy is switched; Coulomb is Eq. 2 up to the cutoff;
//   kCoulEwald     only the LJ energy is switched; Coulomb is the real-space term of an
//                  Ewald sum, k q_i q_j erfc(alpha r) / r, the rest of it being summed in
//                  reciprocal space beyond the short-range kernel.
constexpr int kCoulSwitched = 0, kCoulPlain = 1, kCoulEwald = 2;

// Pair force factor f (F_i = f r_ij) and pair energy e at squared distance u.
// c12 = 4 eps s^12, c6 = 4 eps s^6 (Eq. 1: A = 12 c12, B = 6 c6); qq = k q_i q_j (Eq. 2).
// The switch in s = 1 - t = clamp((rc^2 - u)/(rc^2 - rs^2), 0, 1): S = s^2 (3 - 2s) =
// (1-t)^2 (1+2t), and g = 12 s (1-s) / (rc^2 - rs^2) = -2 dS/du. rc^2 - u is exact near the
// cutoff (Sterbenz), so s, S and g keep their relative accuracy where they are small; and
// rc^2 - u <= 0 exactly for u >= rc^2, so with the whole energy switched a pair at or past
// the cutoff gets s = 0 and adds exactly zero force and energy. inv_sw is
// 1/(rc^2 - rs^2), or with the switch off 2^100 (s = 1 for every u < rc^2; sw12 = 0).
// Ewald: e_C = qq erfc(a r)/r and -(1/r) de_C/dr =
// qq (erfc(a r)/r + (2a/sqrt(pi)) exp(-a^2 u)) / u, with ew = (a, 2a/sqrt(pi)).
template <int kCoul, typename Real>
__device__ inline Real pair_f(Real u, Real c12, Real c6, Real qq, Real rc2, Real inv_sw,
                              Real sw12, Real& e, V2<Real> ew = {}) {
  Real rinv, s;
  if constexpr (sizeof(Real) == 4) {
    rinv = __builtin_amdgcn_rsqf(u);
    s = __builtin_amdgcn_fmed3f((rc2 - u) * inv_sw, 0.f, 1.f);
  } else {
    rinv = 1.0 / sqrt(u);
    s = fmin(fmax((rc2 - u) * inv_sw, 0.0), 1.0);
  }
  const Real r2 = rinv * rinv;
  const Real r6 = r2 * r2 * r2;
  const Real c6r6 = c6 * r6;
  const Real elj = mad(c12 * r6, r6, -c6r6);        // c12/r^12 - c6/r^6
  const Real x6 = mad(Real(2), elj, c6r6);          // (12 c12/r^12 - 6 c6/r^6) / 6
  const Real ec = qq * rinv;
  const Real s2 = s * s;
  const Real S = s2 * mad(Real(-2), s, Real(3));   // (1-t)^2 (1+2t)
  const Real g = (s - s2) * sw12;                  // 12 t (1-t) / (rc^2 - rs^2)
  if (kCoul == kCoulSwitched) {
    const Real et = elj + ec;
    e = S * et;
    return mad(g, et, S * mad(Real(6), x6, ec) * r2);
  }
  if (kCoul == kCoulEwald) {
    const Real ar = ew.x * (u * rinv);
    Real sc, ex;
    if constexpr (sizeof(Real) == 4) {
      sc = erfcf(ar);
      ex = expf(-ar * ar);
    } else {
      sc = erfc(ar);
      ex = exp(-ar * ar);
    }
    const Real es = ec * sc;                          // qq erfc(a r) / r
    e = mad(S, elj, es);
    return mad(g, elj, mad(Real(6) * S, x6, mad(qq * ew.y, ex, es)) * r2);
  }
  e = mad(S, elj, ec);
  return mad(g, elj, mad(Real(6) * S, x6, ec) * r2);
}

// Four 16-bit LDS stores of v, store i by the lanes set in m_i only, to byte addresses
// relative to the start of LDS (the dynamic block starts there: the kernel has no static
// LDS). The exec mask is narrowed for each store and restored, so no per-lane select is
// needed and the addresses need no further add. LDS operations of one wave complete in order, so the
// compiler's own waits on later LDS reads stay valid.
// (n << 1) + b in one scalar instruction
__device__ inline uint32_t lshl1_add(uint32_t n, uint32_t b) {
  uint32_t r;
  __asm__("s_lshl1_add_u32 %0, %1, %2" : "=s"(r) : "s"(n), "s"(b) : "scc");
  return r;
}

__device__ inline void lds_store_u16_lanes4(uint32_t a0, uint32_t a1, uint32_t a2, uint32_t a3,
                                            uint32_t v, unsigned long long m0,
                                            unsigned long long m1, unsigned long long m2,
                                            unsigned long long m3) {
  unsigned long long saved;
  __asm__ volatile(
      "s_mov_b64 %0, exec\n\t"
      "s_and_b64 exec, %0, %6\n\t"
      "ds_write_b16 %1, %5\n\t"
      "s_and_b64 exec, %0, %7\n\t"
      "ds_write_b16 %2, %5\n\t"
      "s_and_b64 exec, %0, %8\n\t"
      "ds_write_b16 %3, %5\n\t"
      "s_and_b64 exec, %0, %9\n\t"
      "ds_write_b16 %4, %5\n\t"
      "s_mov_b64 exec, %0"
      : "=&s"(saved)
      : "v"(a0), "v"(a1), "v"(a2), "v"(a3), "v"(v), "s"(m0), "s"(m1), "s"(m2), "s"(m3)
      : "memory", "scc");
}

// kClamp: the whole energy is switched and the switch is on, so lanes that must add
// nothing (a partial batch, the home atom itself) get u = kBigU instead of masks on f
// and e, and pairs beyond the cutoff need no test (the switch variable s clamps to 0).
// kDiag: count filter passes, cutoff passes and filtered slots (MD_DIAG_COUNTERS).
// kHalf: the half shell (64-bit fixed-point sums only). kDrain: force batches per drain.
template <typename Real, bool kHalf, int kCoul, bool kClamp, bool kDiag, int kDrain>
__device__ __attribute__((always_inline)) inline bool pair_fs(const SysArgs<Real>& a, int cap,
                                                              int64_t cellA, int part) {
  extern __shared__ __attribute__((aligned(16))) unsigned char s_dyn[];
  constexpr bool kF32 = sizeof(Real) == 4;
  constexpr int kImg = kHalf ? 14 : 27;   // neighbour images
  constexpr int kFifo = fifo_entries(kDrain);
  constexpr int kWaveFifo = kQ * kFifo;
  constexpr uint32_t kS = sizeof(V4<Real>);   // bytes per staged atom record
  constexpr int kAW = kAccWords<Real>;
  using R4 = V4<Real>;
  using R2 = V2<Real>;
  const Lds LL = lds_layout<Real>(cap, a.n_types, kHalf, kDiag, kDrain);
  Hdr& H = *reinterpret_cast<Hdr*>(s_dyn + LL.hdr);
  uint16_t* sFifo = reinterpret_cast<uint16_t*>(s_dyn + LL.fifo);
  R2* sLJ = reinterpret_cast<R2*>(s_dyn + LL.lj);
  R4* sF = reinterpret_cast<R4*>(s_dyn + LL.f4);
  Real* sQ = reinterpret_cast<Real*>(s_dyn + LL.q);
  [[maybe_unused]] int* sT = reinterpret_cast<int*>(s_dyn + LL.typ);   // float64: types
  long long* sJ = reinterpret_cast<long long*>(s_dyn + LL.jacc);   // [cap][3][kAW], half
  int* sJn = reinterpret_cast<int*>(s_dyn + LL.jcnt);               // [cap], half + counters

  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nt = a.n_types;
  // float32: low bits of a staged c_j that carry the atom's type
  [[maybe_unused]] const uint32_t tmask =
      nt > 1 ? (2u << (31 - __builtin_clz((unsigned)(nt - 1)))) - 1u : 0u;
  constexpr bool diag = kDiag;
  const bool f32 = kF32 && !kHalf && (a.flags & MD_ACCUM_F32_ATOMIC) != 0;
  const Real rc2 = a.rc2, sw12 = Real(12) * a.inv_sw;
  const Real inv_sw = a.inv_sw > Real(0) ? a.inv_sw : Real(0x1p100);   // off: s = 1 below rc^2
  const R2 ew = mk2<Real>(a.ewald_alpha, a.ewald_alpha * Real(1.1283791670955126));   // 2/sqrt(pi)
  const Real L0 = a.L[0], L1 = a.L[1], L2 = a.L[2];
  const int ac0 = (int)(cellA % a.nx), ac1 = (int)((cellA / a.nx) % a.ny),
            ac2 = (int)(cellA / ((int64_t)a.nx * a.ny));
  // origin o of the prefilter: the home cell's centre (any nearby point would do)
  const Real O0 = ((Real)ac0 + Real(0.5)) * (L0 / (Real)a.nx);
  const Real O1 = ((Real)ac1 + Real(0.5)) * (L1 / (Real)a.ny);
  const Real O2 = ((Real)ac2 + Real(0.5)) * (L2 / (Real)a.nz);

  for (int e = tid; e < nt * nt; e += kThreads) sLJ[e] = mk2<Real>(a.lj[2 * e], a.lj[2 * e + 1]);
  // FIFO entries past a FIFO's fill level are read by partial force passes (and then
  // ignored): start them as valid indices
  for (int e = tid; e < kNW * kWaveFifo / 2; e += kThreads)
    reinterpret_cast<uint32_t*>(sFifo)[e] = 0u;
  const int sA = a.start[cellA];
  const int nA = a.start[cellA + 1] - sA;

  // image table and segments (wave 0; lane l < 2 kImg = half l & 1 of image l >> 1).
  // Pieces are ordered by (shift class, dz, dy, z half, dx), the shift class being the set
  // of axes along which the image lies at +L (grp): the pieces of one (dy, dz) row, one
  // z half and one shift class form a segment, sorted in x because each half of a cell is
  // and the cells follow each other in x. The half shell puts the home image's two halves
  // first, as segments of their own: its neighbour-list positions 0 .. nA-1 are then the
  // home atoms in their sorted order, which the j > i rule compares.
  if (tid < 64) {
    const int m = lane >> 1, h = lane & 1;
    const bool act = lane < 2 * kImg;
    const int nd[3] = {a.nx, a.ny, a.nz};
    const int ac[3] = {ac0, ac1, ac2};
    int grp = 0, jsh = 0, st0 = 0, cnt = 0, n0 = 0, key = 1 << 20, ox = 0;
    int io[3] = {0, 0, 0};   // the image's cell offset
    if (act) {
      for (int d = 0; d < 3; ++d) io[d] = kHalf ? c_himg[m][d] : c_img[m][d];
      int b[3];
      for (int d = 0; d < 3; ++d) {
        b[d] = ac[d] + io[d];
        if (b[d] >= nd[d]) {
          b[d] -= nd[d];
          grp |= 1 << d;
        } else if (b[d] < 0) {
          b[d] += nd[d];
          jsh |= 1 << d;
        }
      }
      const int64_t cb = ((int64_t)b[2] * a.ny + b[1]) * a.nx + b[0];
      st0 = a.start[cb];
      cnt = a.start[cb + 1] - st0;
      n0 = a.zsplit[cb];
      key = (grp * 9 + (io[1] + 1) + 3 * (io[2] + 1)) * 2 + h;
      if (kHalf) key = m == 0 ? h : key + 2;
      ox = io[0];
    }
    const int pc = act ? (h ? cnt - n0 : n0) : 0;   // atoms of this piece
    int off = 0, seg_len = 0, tot = 0;
    bool head = act;
    for (int l2 = 0; l2 < 2 * kImg; ++l2) {
      const int km = __builtin_amdgcn_readlane(key, l2);
      const int cm = __builtin_amdgcn_readlane(pc, l2);
      const int xm = __builtin_amdgcn_readlane(ox, l2);
      const bool same = km == key;
      off += (km < key || (same && xm < ox)) ? cm : 0;
      seg_len += same ? cm : 0;
      if (same && xm < ox) head = false;
      tot += cm;
    }
    // a head (the first piece of its segment) is numbered by the heads with smaller keys
    const unsigned long long heads = __builtin_amdgcn_ballot_w64(head);
    int seg_idx = 0;
    for (int l2 = 0; l2 < 2 * kImg; ++l2) {
      const int km = __builtin_amdgcn_readlane(key, l2);
      seg_idx += (((heads >> l2) & 1ull) && km < key) ? 1 : 0;
    }
    if (act) {
      H.img[m].off[h] = off;
      if (h == 0) {
        H.img[m].start = st0;
        H.img[m].count = cnt;
        H.img[m].n0 = n0;
        H.img[m].grp = grp;
        H.img[m].jsh = jsh;
      }
      if (head) {
        const float wy = (float)L1 / (float)a.ny, wz = (float)L2 / (float)a.nz;
        Seg& sg_ = H.seg[seg_idx];
        sg_.begin = off;
        sg_.end = off + seg_len;
        sg_.grp = grp;
        sg_.y0 = (float)(ac1 + io[1]) * wy;
        sg_.y1 = (float)(ac1 + io[1] + 1) * wy;
        sg_.z0 = ((float)(ac2 + io[2]) + 0.5f * (float)h) * wz;
        sg_.z1 = ((float)(ac2 + io[2]) + 0.5f * (float)(h + 1)) * wz;
      }
    }
    int ml = head ? seg_len : 0;
    for (int s2 = 32; s2 > 0; s2 >>= 1) ml = max(ml, __shfl_xor(ml, s2));
    if (lane == 0) {
      H.n_seg = __builtin_popcountll(heads);
      H.total = tot;
      H.done = 0;
      H.esum[0] = H.esum[1] = 0;
      int it = 0;
      while ((1 << it) <= ml) ++it;   // steps of a lower_bound over ml elements
      H.iters = it;
    }
  }
  __syncthreads();

  const int total = H.total;
  const int n_seg = H.n_seg;
  const int iters = H.iters;
  const int n_grp_q = (nA + kQ - 1) / kQ;
  // this workgroup's share of the home cell: groups part, part + n_split, part + 2 n_split, ..
  const int n_split = a.fs_split;
  // largest home-side partial of one slice (see kAccRange)
  const float home_max = (kHalf ? kAccRange - 14.f * (float)a.fs_split * kNbrPartialMax : kAccRange) /
                         (float)max(1, (total + cap - 1) / cap);
  const Real R = vsqrt(rc2) + Real(kWin);
  // energy: float32 in units of 2^-24 kcal/mol; float64 two-word (e_fix, e_lo): exact,
  // order-independent sums
  long long e_fix = 0;
  [[maybe_unused]] long long e_lo = 0;
  unsigned long long pass_count = 0, filt_count = 0, slot_count = 0, lane_count = 0;
  uint32_t st = 0;
  uint16_t* fifo = sFifo + w * kWaveFifo;
  // LDS byte address where FIFO k of this wave starts: fk0 + 2 k kFifo
  const uint32_t fk0 = (uint32_t)(LL.fifo + 2 * w * kWaveFifo);

  for (int P0 = 0; P0 < total; P0 += cap) {
    const int P1 = min(total, P0 + cap);
    // stage the neighbour-list slice [P0, P1): wave w copies images w and w + 16 (both z
    // halves, to their two segments), issuing all loads of up to 4 x 64 atoms before the
    // LDS stores; the half shell also clears the slots' accumulators
    for (int m = w; m < kImg; m += kNW) {
      const Img im = H.img[m];
      // o_g = o - h: the origin in this image's frame
      const Real og0 = O0 - ((im.grp & 1) ? L0 : Real(0));
      const Real og1 = O1 - ((im.grp & 2) ? L1 : Real(0));
      const Real og2 = O2 - ((im.grp & 4) ? L2 : Real(0));
      for (int e0 = 0; e0 < im.count; e0 += 4 * 64) {
        P4<Real> v[4];
        int tv[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int e = e0 + 64 * r + lane;
          const int src = im.start + min(e, im.count - 1);
          v[r] = a.pos[src];
          tv[r] = a.type[src];
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int e = e0 + 64 * r + lane;
          const int dst = e < im.n0 ? im.off[0] + e : im.off[1] + (e - im.n0);
          if (e < im.count && dst >= P0 && dst < P1) {
            const Real x = (im.jsh & 1) ? v[r].x - L0 : v[r].x;
            const Real y = (im.jsh & 2) ? v[r].y - L1 : v[r].y;
            const Real z = (im.jsh & 4) ? v[r].z - L2 : v[r].z;
            const Real rx = x - og0, ry = y - og1, rz = z - og2;
            const Real cj = mad(rz, rz, mad(ry, ry, rx * rx));
            if constexpr (kF32) {
              // c_j with its low mantissa bits (as many as the types need, at most 6)
              // replaced by the type: under 64 ulps of c_j, at most 1.6e-2 A^2 for the
              // largest cells (18 A), well inside the prefilter's margin
              const uint32_t w4 = (__float_as_uint(cj) & ~tmask) | (uint32_t)tv[r];
              sF[dst - P0] = mk4(x, y, z, __uint_as_float(w4));
            } else {
              sF[dst - P0] = mk4(x, y, z, cj);
              sT[dst - P0] = tv[r];
            }
            sQ[dst - P0] = v[r].w;
            if (kHalf) {
#pragma unroll
              for (int c = 0; c < 3 * kAW; ++c) sJ[3 * kAW * (dst - P0) + c] = 0;
              if (kDiag) sJn[dst - P0] = 0;
            }
          }
        }
      }
    }
    if (tid == 0) H.next = 0;
    __syncthreads();

    // segment table in registers, clipped to this slice: lane l holds segment l, or, when
    // there are at most 32 segments, segment l & 31, so that lanes l and l + 32 can search
    // the two ends of segment l's x-window at once
    const bool split = n_seg <= 32;
    const int sl = split ? (lane & 31) : lane;
    int sb = 0, se = 0, sg = 0;
    if (sl < n_seg) {
      sb = max(H.seg[sl].begin, P0) - P0;
      se = max(min(H.seg[sl].end, P1) - P0, sb);
      sg = H.seg[sl].grp;
    }
    // first position p in [sb, se) of this lane's segment with x >= key (se if none): a
    // power-of-two search over byte addresses, 2^iters > se - sb, each probe clamped to
    // the segment's last atom (a probe past it compares that atom instead, and the result
    // is clamped to se)
    const uint32_t f4b = (uint32_t)LL.f4;
    auto lower_bound = [&](Real key) __attribute__((always_inline)) {
      const Real k = se > sb ? key : Real(-INFINITY);   // an empty segment probes nothing
      uint32_t a = f4b + kS * (uint32_t)sb - kS;          // byte address of the last atom < key
      const uint32_t last = f4b + kS * (uint32_t)se - kS;
      for (int it = iters - 1; it >= 0; --it) {
        const uint32_t t = a + (kS << it);
        const Real xq = *reinterpret_cast<const __attribute__((address_space(3))) Real*>(
            (uintptr_t)min(t, last));   // LDS byte address (the dynamic block starts at 0)
        a = xq < k ? t : a;
      }
      return min((int)((a + kS - f4b) / kS), se);
    };

    while (true) {
      int o = 0;
      if (lane == 0) o = atomicAdd(&H.next, 1);
      o = part + n_split * __builtin_amdgcn_readfirstlane(__shfl(o, 0));
      if (o >= n_grp_q) break;
      const int ib = kQ * o;
      const int nv = min(kQ, nA - ib);   // home atoms present in this group

      // home atom k of the group in the frame of no shift (xi, yi, zi) and in that of the
      // current segment (xs, ys, zs; its shift class cur_g), its prefilter constants (ax,
      // ay, az; thb, and thr, the threshold in the current frame), k q and its row of the
      // type-pair table, loaded as the in-cell sort wrote them; an absent atom (past nv)
      // repeats the last one with ax = 0 and thb = -1, which c_j >= 0 never passes
      Real xi[kQ], yi[kQ], zi[kQ], thb[kQ];   // frame of no shift
      Real xs[kQ], ys[kQ], zs[kQ], thr[kQ], kq[kQ], fx[kQ], fy[kQ], fz[kQ];
      Real ax[kQ], ay[kQ], az[kQ];
      int row[kQ];
      uint32_t fb[kQ];   // byte address of the next free slot of FIFO k
      uint32_t fl[kQ];   // fb[k] at which FIFO k holds a full drain
      unsigned cnt[kQ];
      Real xmin = 0, xmax = 0, ymin = 0, ymax = 0, zmin = 0, zmax = 0;
#pragma unroll
      for (int k = 0; k < kQ; ++k) {
        const int s = sA + ib + min(k, nv - 1);
        const P4<Real> p = a.pos[s];
        const P4<Real> h0 = a.hpre[2 * (int64_t)s], h1 = a.hpre[2 * (int64_t)s + 1];
        xi[k] = p.x;
        yi[k] = p.y;
        zi[k] = p.z;
        ax[k] = h0.x;
        ay[k] = h0.y;
        az[k] = h0.z;
        thb[k] = h0.w;
        kq[k] = h1.x;
        row[k] = slot_to_int(h1.y);
        xmin = k == 0 ? p.x : vmin(xmin, p.x);
        xmax = k == 0 ? p.x : vmax(xmax, p.x);
        ymin = k == 0 ? p.y : vmin(ymin, p.y);
        ymax = k == 0 ? p.y : vmax(ymax, p.y);
        zmin = k == 0 ? p.z : vmin(zmin, p.z);
        zmax = k == 0 ? p.z : vmax(zmax, p.z);
        fx[k] = fy[k] = fz[k] = Real(0);
        fb[k] = fk0 + 2u * (uint32_t)(k * kFifo);
        fl[k] = fb[k] + 2u * (uint32_t)(64 * kDrain);
        cnt[k] = 0;
      }
      if (nv < kQ) {
#pragma unroll
        for (int k = 1; k < kQ; ++k) {
          if (k >= nv) {
            ax[k] = ay[k] = az[k] = Real(0);
            thb[k] = Real(-1);
          }
        }
      }
#pragma unroll
      for (int k = 0; k < kQ; ++k) {
        xs[k] = xi[k];
        ys[k] = yi[k];
        zs[k] = zi[k];
        thr[k] = thb[k];
      }
      Real e_lane = 0;
      // the largest |F_j| component |f dx| handed to the neighbour side (float32: as
      // |f| times the largest |dx|)
      Real jmax = 0;

      // x-window of every segment: [lo, hi) of segment s with x in [min x_i - w, max x_i + w)
      // in the segment's frame (two lower_bound searches, in lanes s and s + 32 when the
      // segments fit 32 lanes, else both in lane s), where w^2 = R^2 - gy^2 - gz^2 and gy,
      // gz are the gaps between the group's bounding box and the segment's slab (less
      // 1e-3 A for atoms binned at a face by rounding)
      int wlo, whi;
      {
        // the segment's slab, read again for every group (registers are scarce)
        const Seg& sgl = H.seg[sl < n_seg ? sl : 0];
        const float4 slab = make_float4(sgl.y0, sgl.y1, sgl.z0, sgl.z1);
        const Real gy = vmax(vmax((Real)slab.x - ymax, ymin - (Real)slab.y) - Real(kWin), Real(0));
        const Real gz = vmax(vmax((Real)slab.z - zmax, zmin - (Real)slab.w) - Real(kWin), Real(0));
        const Real w2 = mad(R, R, -mad(gz, gz, gy * gy));
        const Real hw = w2 > Real(0) ? wsqrt(w2) : Real(-1);
        const Real hx = (sg & 1) ? L0 : Real(0);
        // a segment out of reach gets the empty window [sb, sb)
        const Real xlo = w2 > Real(0) ? (xmin - hx) - hw : Real(-INFINITY);
        const Real xhi = w2 > Real(0) ? (xmax - hx) + hw : Real(-INFINITY);
        if (split) {
          // lane s: start of segment s's window; lane s + 32: its end
          wlo = lower_bound(lane < 32 ? xlo : xhi);
          whi = wlo;
        } else {
          wlo = lower_bound(xlo);
          whi = lower_bound(xhi);
        }
      }

      // entries in FIFO k
      auto fill = [&](int k) __attribute__((always_inline)) {
        return (int)((fb[k] - fk0) >> 1) - k * kFifo;
      };
      // type of a staged atom
      auto type_of = [&](int jl, const R4& pj) __attribute__((always_inline)) {
        if constexpr (kF32) return (int)(__float_as_uint(pj.w) & tmask); else return sT[jl];
      };
      // the force on home atom k from one lane's FIFO entry j: the exact distance in the
      // current frame, the strict cutoff and the force; `in` is false for lanes past the
      // FIFO's fill level. The full shell's u > 0 drops the home atom itself; the half
      // shell never pairs an atom with itself (j > i in the home image). The half shell
      // adds -F to neighbour j's accumulator as well (zero for lanes that add nothing):
      // float32 in units of 2^-24 kcal/mol/A (-f dx, exact in float64, rounded once to a
      // multiple of 2^-24), float64 as a two-word fixed-point value.
      auto pair_lane = [&](int k, int jl, const R4& pj, Real qj, const R2& lj,
                           bool in) __attribute__((always_inline)) {
        const Real dx = xs[k] - pj.x, dy = ys[k] - pj.y, dz = zs[k] - pj.z;
        Real u = dist2(dx, dy, dz);
        Real e, f;
        if (kClamp) {
          u = (in && (kHalf || u > Real(0))) ? u : Real(kBigU);
          f = pair_f<kCoul>(u, lj.x, lj.y, kq[k] * qj, rc2, inv_sw, sw12, e, ew);
          if (diag) cnt[k] += __builtin_popcountll(__builtin_amdgcn_ballot_w64(u < rc2));
          if (kHalf && diag && u < rc2) atomicAdd(&sJn[jl], 1);
        } else {
          const bool lv = in && u < rc2 && u > Real(0);
          f = pair_f<kCoul>(u, lj.x, lj.y, kq[k] * qj, rc2, inv_sw, sw12, e, ew);
          f = lv ? f : Real(0);
          e = lv ? e : Real(0);
          if (diag) cnt[k] += __builtin_popcountll(__builtin_amdgcn_ballot_w64(lv));
          if (kHalf && diag && lv) atomicAdd(&sJn[jl], 1);
        }
        fx[k] = mad(f, dx, fx[k]);
        fy[k] = mad(f, dy, fy[k]);
        fz[k] = mad(f, dz, fz[k]);
        e_lane += e;
        if (kHalf) {
          if constexpr (kF32) {
            const double nf = -(double)f;
            const float m3 = fmaxf(fmaxf(fabsf(dx), fabsf(dy)), fabsf(dz));   // one v_max3
            jmax = fmaxf(jmax, fabsf(f * m3));
            long long* d = sJ + 3 * jl;
            lds_add(d, round_prod_2m24(nf, dx));
            lds_add(d + 1, round_prod_2m24(nf, dy));
            lds_add(d + 2, round_prod_2m24(nf, dz));
          } else {
            const double p3[3] = {-f * dx, -f * dy, -f * dz};
            long long* d = sJ + 6 * jl;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              jmax = fmax(jmax, fabs(p3[c]));
              const Fix2 q2 = to_fix2(fmin(fmax(p3[c], -1.0e9), 1.0e9));
              lds_add(d + 2 * c, q2.hi);
              lds_add(d + 2 * c + 1, q2.lo);
            }
          }
        }
      };
      // dense force passes over the first 64 kDrain entries of FIFO k, every lane busy; all
      // LDS reads of the kDrain batches precede the arithmetic. The remainder (fewer than
      // 64 entries) moves to the front.
      auto force = [&](int k) __attribute__((always_inline)) {
        int jj[kDrain], tj[kDrain];
        R4 pj[kDrain];
        Real qj[kDrain];
        R2 lj[kDrain];
#pragma unroll
        for (int b = 0; b < kDrain; ++b) jj[b] = fifo[k * kFifo + 64 * b + lane];
        if (diag) lane_count += 64 * kDrain;
#pragma unroll
        for (int b = 0; b < kDrain; ++b) {
          pj[b] = sF[jj[b]];
          qj[b] = sQ[jj[b]];
          tj[b] = type_of(jj[b], pj[b]);
        }
#pragma unroll
        for (int b = 0; b < kDrain; ++b) lj[b] = sLJ[row[k] + tj[b]];
#pragma unroll
        for (int b = 0; b < kDrain; ++b) pair_lane(k, jj[b], pj[b], qj[b], lj[b], true);
        const int c = 64 * kDrain;
        const int rem = fill(k) - c;
        if (rem > 0) {
          uint16_t v = 0;
          if (lane < rem) v = fifo[k * kFifo + c + lane];
          if (lane < rem) fifo[k * kFifo + lane] = v;
        }
        fb[k] = fk0 + 2u * (uint32_t)(k * kFifo + rem);
      };
      // every entry left in the FIFOs, one 64-lane pass at a time (the home side is about
      // to change frame, or the group is done)
      auto flush = [&]() __attribute__((always_inline)) {
#pragma unroll
        for (int k = 0; k < kQ; ++k) {
          const int n = fill(k);
          for (int off = 0; off < n; off += 64) {
            const int jj = fifo[k * kFifo + off + lane];   // entries past n: valid indices
            if (diag) lane_count += 64;
            const R4 pj = sF[jj];
            const Real qj = sQ[jj];
            const R2 lj = sLJ[row[k] + type_of(jj, pj)];
            pair_lane(k, jj, pj, qj, lj, off + lane < n);
          }
          fb[k] = fk0 + 2u * (uint32_t)(k * kFifo);
        }
      };

      int cur_g = 0;   // the group starts in the frame of no shift
      for (int s = 0; s < n_seg; ++s) {
        int lo = __builtin_amdgcn_readlane(wlo, s);
        const int hi = max(__builtin_amdgcn_readlane(whi, split ? s + 32 : s), lo);
        // half shell, home image (segments 0 and 1, positions = home atom indices): only
        // j > i, so the window starts past the group's first atom, and the first batch
        // drops, for each home atom, the lanes at or before it
        const bool home_seg = kHalf && s < 2;
        if (home_seg) lo = max(lo, ib + 1 - P0);
        if (lo >= hi) continue;
        const int g = __builtin_amdgcn_readlane(sg, s);
        if (g != cur_g) {
          flush();   // the home side changes frame
          cur_g = g;
          const Real hx = (g & 1) ? L0 : Real(0), hy = (g & 2) ? L1 : Real(0),
                     hz = (g & 4) ? L2 : Real(0);
#pragma unroll
          for (int k = 0; k < kQ; ++k) {
            xs[k] = xi[k] - hx;   // exact: such home atoms lie in the last cell of the axis
            ys[k] = yi[k] - hy;
            zs[k] = zi[k] - hz;
            // ax.o_g = ax.o - ax.h (an absent atom keeps thr = -1: its ax is 0)
            thr[k] = thb[k] - (ax[k] * hx + ay[k] * hy + az[k] * hz);
          }
        }
        if (diag) slot_count += (unsigned long long)(hi - lo) * (unsigned long long)nv;
        // se: end of this segment. Lanes in [hi, se) are neighbours of this segment (this
        // frame) past the x-window, farther than r_cut from every home atom of the group:
        // the exact test drops any that the prefilter's margin lets through. Lanes past se
        // belong to another segment (or to the q block, still inside LDS) and are masked.
        const int se_s = __builtin_amdgcn_readlane(se, s);
        for (int jb = lo; jb < hi; jb += 64) {
          const int j = jb + lane;
          const R4 pj = sF[j];
          Real t[kQ];
#pragma unroll
          for (int k = 0; k < kQ; ++k) t[k] = mad(ax[k], pj.x, pj.w);
#pragma unroll
          for (int k = 0; k < kQ; ++k) t[k] = mad(ay[k], pj.y, t[k]);
#pragma unroll
          for (int k = 0; k < kQ; ++k) t[k] = mad(az[k], pj.z, t[k]);
          unsigned long long m[kQ];
#pragma unroll
          for (int k = 0; k < kQ; ++k) m[k] = __builtin_amdgcn_ballot_w64(t[k] < thr[k]);
          if (jb + 64 > se_s) {
            const unsigned long long vm = (1ull << (se_s - jb)) - 1ull;   // se_s - jb < 64
#pragma unroll
            for (int k = 0; k < kQ; ++k) m[k] &= vm;
          }
          if (home_seg && jb + P0 < ib + kQ) {
#pragma unroll
            for (int k = 1; k < kQ; ++k) {
              // lanes 0 .. c-1 hold j <= i = ib + k; c <= k since jb + P0 > ib
              const int c = ib + k + 1 - (jb + P0);
              if (c > 0) m[k] &= ~((1ull << c) - 1ull);
            }
          }
          // passing lanes append at their prefix rank
          uint32_t adr[kQ];
#pragma unroll
          for (int k = 0; k < kQ; ++k) {
            const uint32_t rank = __builtin_amdgcn_mbcnt_hi(
                (unsigned)(m[k] >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m[k], 0u));
            adr[k] = fb[k] + 2u * rank;
          }
#pragma unroll
          for (int k = 0; k < kQ; k += 4)
            lds_store_u16_lanes4(adr[k], adr[k + 1], adr[k + 2], adr[k + 3], (uint32_t)j, m[k],
                                 m[k + 1], m[k + 2], m[k + 3]);
#pragma unroll
          for (int k = 0; k < kQ; ++k) fb[k] = lshl1_add((uint32_t)__builtin_popcountll(m[k]), fb[k]);
          if (diag) {
#pragma unroll
            for (int k = 0; k < kQ; ++k) filt_count += __builtin_popcountll(m[k]);
          }
#pragma unroll
          for (int k = 0; k < kQ; ++k) {
            if (fb[k] >= fl[k]) force(k);
          }
        }
      }
      flush();

      // per home atom and component: the 64 lane partials summed in one fixed order. The
      // two wave halves exchange the sums the other one keeps (lanes l and l ^ 32: home
      // atoms 0, 1 stay in the lower half, 2, 3 in the upper), then the two rows of each
      // half (l and l ^ 16), so that the 16 lanes of row g hold home atom g's three
      // components; a butterfly within the row completes them. Lane 16 g adds atom g's
      // totals to its 64-bit fixed-point sum (exact conversion; with an integer atomic in
      // the half shell, where other workgroups add to the same atom) or float32 sum.
      static_assert(kQ == 4, "one 16-lane row per home atom");
      Real r[3 * kQ];
#pragma unroll
      for (int k = 0; k < kQ; ++k) {
        r[3 * k] = fx[k];
        r[3 * k + 1] = fy[k];
        r[3 * k + 2] = fz[k];
      }
      Real r3[3];
      if constexpr (kF32) {
        // Both exchanges are register swaps between lane groups (v_permlane32_swap: lanes
        // 32-63 of the first operand with lanes 0-31 of the second; v_permlane16_swap: the
        // odd 16-lane rows of the first with the even rows of the second). After the swap
        // the first operand holds the lane's kept value in the lower group and the
        // partner's in the upper one, the second operand the reverse, so their sum is the
        // same two terms as keep + partner's give (float addition commutes exactly). The
        // results are read by value: a bit cast applied to an element of the returned
        // vector reads element 0 for both with this compiler.
        float r6[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) {
          const auto sw = __builtin_amdgcn_permlane32_swap(__float_as_uint(r[i]),
                                                           __float_as_uint(r[i + 6]), false, false);
          r6[i] = __uint_as_float(sw[0]) + __uint_as_float(sw[1]);
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          const auto sw = __builtin_amdgcn_permlane16_swap(__float_as_uint(r6[i]),
                                                           __float_as_uint(r6[i + 3]), false, false);
          r3[i] = __uint_as_float(sw[0]) + __uint_as_float(sw[1]);
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) r3[i] = rowsum16(r3[i]);
      } else {
        // the same order with lane shuffles: own + partner's term at each step
        const bool upper = lane >= 32, odd_row = (lane & 16) != 0;
        double r6[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) {
          const double keep = upper ? r[i + 6] : r[i];
          const double give = upper ? r[i] : r[i + 6];
          r6[i] = keep + __shfl_xor(give, 32);
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          const double keep = odd_row ? r6[i + 3] : r6[i];
          const double give = odd_row ? r6[i] : r6[i + 3];
          r3[i] = keep + __shfl_xor(give, 16);
        }
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int sft = 1; sft < 16; sft <<= 1) r3[i] += __shfl_xor(r3[i], sft);
      }
      {
        const int kr = lane >> 4;   // this row's home atom
        if ((lane & 15) == 0 && kr < nv) {
          const int64_t s = sA + ib + kr;
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            if (f32) {
              float* dst = &a.facc[(int64_t)c * a.n + s];
              *dst = P0 == 0 ? (float)r3[c] : *dst + (float)r3[c];
            } else {
              // one of the slice count's home-side partials of this atom: within its share
              // of the fixed point's range (kAccRange)
              if (!(fabs(r3[c]) < (Real)home_max)) st |= MD_STATUS_FIXED_OVERFLOW;
              if constexpr (kF32) {
                const long long qv = to_fixed(r3[c], st);
                long long* dst = &a.acc64[(int64_t)c * a.n + s];
                if (kHalf)
                  global_add(dst, qv);
                else
                  *dst = P0 == 0 ? qv : *dst + qv;
              } else {
                const Fix2 q2 = to_fix2(fmin(fmax(r3[c], -1.0e10), 1.0e10));
                long long* dh = &a.acc64[(int64_t)c * a.n + s];
                long long* dl = &a.acc64[(int64_t)(3 + c) * a.n + s];
                if (kHalf) {
                  global_add(dh, q2.hi);
                  global_add(dl, q2.lo);
                } else {
                  *dh = P0 == 0 ? q2.hi : *dh + q2.hi;
                  *dl = P0 == 0 ? q2.lo : *dl + q2.lo;
                }
              }
            }
          }
          if (diag) {
            unsigned ck = cnt[0];
#pragma unroll
            for (int k = 1; k < kQ; ++k) ck = kr == k ? cnt[k] : ck;
            int* dst = &a.paircount[a.n + s];
            if (kHalf)
              atomicAdd(dst, (int)ck);
            else
              *dst = P0 == 0 ? (int)ck : *dst + (int)ck;
          }
        }
      }
#pragma unroll
      for (int k = 0; k < kQ; ++k) pass_count += k < nv ? cnt[k] : 0u;
      if constexpr (kF32) {
        // the group's lane energy in 64-bit fixed point (exact scaling by 2^24, then one
        // rounding), so the workgroup total does not depend on which wave took which group
        const float v = e_lane * 16777216.0f;
        if (!(fabsf(v) < 4.6116860184273879e18f)) st |= MD_STATUS_FIXED_OVERFLOW;
        else e_fix += round_to_i64((double)v);
        if (kHalf && !(jmax < kNbrPartialMax)) st |= MD_STATUS_FIXED_OVERFLOW;
      } else {
        if (!(fabs(e_lane) < 1.0e9)) {
          st |= MD_STATUS_FIXED_OVERFLOW;
        } else {
          const Fix2 q2 = to_fix2(e_lane);
          e_fix += q2.hi;
          e_lo += q2.lo;
        }
        if (kHalf && !(jmax < (double)kNbrPartialMax)) st |= MD_STATUS_FIXED_OVERFLOW;
      }
    }
    __syncthreads();
    if (kHalf) {
      // neighbour-side sums of this slice to the per-atom sums (wave w: images w, w + 16)
      for (int m = w; m < kImg; m += kNW) {
        const Img im = H.img[m];
        for (int e = lane; e < im.count; e += 64) {
          const int dst = e < im.n0 ? im.off[0] + e : im.off[1] + (e - im.n0);
          if (dst < P0 || dst >= P1) continue;
          const int64_t src = im.start + e;
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            if constexpr (kF32) {
              // units of 2^-24 to the sums' 2^-28, each partial below 2^27 kcal/mol/A (2^51
              // units, kNbrPartialMax)
              const long long v = sJ[3 * (dst - P0) + c];
              constexpr long long kLim = (long long)kNbrPartialMax << 24;
              if (v >= kLim || v < -kLim) st |= MD_STATUS_FIXED_OVERFLOW;
              else if (v != 0)
                global_add(&a.acc64[(int64_t)c * a.n + src],
                           (long long)((unsigned long long)v << 4));
            } else {
              // two words, the low one reduced into [0, 2^52) so that the 14 neighbour-side
              // partials of an atom cannot wrap it; each partial below 2^27 kcal/mol/A
              const Fix2 v = normalize2(sJ[6 * (dst - P0) + 2 * c], sJ[6 * (dst - P0) + 2 * c + 1]);
              constexpr long long kLim = (long long)kNbrPartialMax << 20;
              if (v.hi >= kLim || v.hi < -kLim) {
                st |= MD_STATUS_FIXED_OVERFLOW;
              } else {
                if (v.hi != 0) global_add(&a.acc64[(int64_t)c * a.n + src], v.hi);
                if (v.lo != 0) global_add(&a.acc64[(int64_t)(3 + c) * a.n + src], v.lo);
              }
            }
          }
          if (kDiag) {
            const int v = sJn[dst - P0];
            if (v != 0) atomicAdd(&a.paircount[a.n + src], v);
          }
        }
      }
      // the next slice clears the accumulators; after the last one nothing waits here, so
      // the workgroup can end while its atomics are still on their way
      if (P0 + cap < total) __syncthreads();
    }
  }

  // workgroup energy (the full shell saw each pair from both atoms) as an exact integer
  // sum: each wave adds its lanes, then its total into the workgroup's LDS words (integer
  // adds: the result does not depend on their order); the last wave to do so stores the
  // total, which the finalize kernel adds to the others as integers too. No barrier: a
  // wave's LDS operations complete in order, so the last wave's read follows every other
  // wave's add.
  bool last;
  {
    long long v0, v1 = 0;
    if constexpr (kF32) {
      v0 = e_fix;
    } else {
      const Fix2 v = normalize2(e_fix, e_lo);   // low words below 2^52: 1024 of them fit
      v0 = v.hi;
      v1 = v.lo;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      v0 += __shfl_xor(v0, off);
      if constexpr (!kF32) v1 += __shfl_xor(v1, off);
    }
    int rank = 0;
    if (lane == 0) {
      lds_add(&H.esum[0], v0);
      if constexpr (!kF32) lds_add(&H.esum[1], v1);
      rank = __hip_atomic_fetch_add(&H.done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    last = __builtin_amdgcn_readfirstlane(__shfl(rank, 0)) == kNW - 1;
    if (last && lane == 0) {
      const int64_t slot = part * a.n_cells + cellA;
      long long* ep = reinterpret_cast<long long*>(a.epart);
      if constexpr (kF32) {
        ep[slot] = __hip_atomic_load(&H.esum[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      } else {
        const Fix2 s2 = normalize2(
            __hip_atomic_load(&H.esum[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP),
            __hip_atomic_load(&H.esum[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
        ep[2 * slot] = s2.hi;
        ep[2 * slot + 1] = s2.lo;
      }
    }
  }
  if (st) atomicOr(&a.hdr->status, st);
  if (diag && lane == 0) {
    // candidates of Algorithm 1: every (home atom, other neighbour-list atom), counted
    // from both atoms in the full shell (halved after the kernel) and once in the half
    // shell; the neighbour slots this kernel actually filtered come separately
    if (w == 0 && part == 0) {
      const unsigned long long nA_ = (unsigned long long)nA;
      const unsigned long long cand =
          kHalf ? nA_ * (nA_ - 1) / 2 + nA_ * (unsigned long long)(total - nA)
                : nA_ * (unsigned long long)(total - 1);
      atomicAdd(&a.hdr->diag[0], cand);
    }
    atomicAdd(&a.hdr->diag[1], filt_count);
    atomicAdd(&a.hdr->diag[2], pass_count);
    atomicAdd(&a.hdr->diag[3], slot_count);
    atomicAdd(&a.hdr->diag[4], lane_count);
  }
  return last;   // this wave is the workgroup's last to finish
}

// The workgroup's time for its home cell (constant 100 MHz clock) goes to cost[cell]: the
// binning of the next evaluation on this grid (of at most 1024 cells) launches the cells
// longest first by it (measurement-based load balancing; atom counts stand in on the
// first evaluation and on larger grids). The first workgroup marks the costs valid for
// this grid.
// The same workgroup also adds its shader-clock cycles (s_memtime) and its 100 MHz ticks
// to the header's two clock sums: their ratio is the clock the kernel ran at, weighted by
// workgroup time. Called by lane 0 of the workgroup's last wave to finish.
template <typename Real>
__device__ inline void record_cost(const SysArgs<Real>& a, int64_t cell, int part, uint64_t t0,
                                   uint64_t c0, bool first) {
  const uint64_t dc = __builtin_amdgcn_s_memtime() - c0;
  const uint64_t dt = __builtin_amdgcn_s_memrealtime() - t0;
  if (part == 0) a.cost[cell] = dt < 0xffffffffull ? (uint32_t)dt : 0xffffffffu;
  atomicAdd(&a.hdr->clock[0], (unsigned long long)dc);
  atomicAdd(&a.hdr->clock[1], (unsigned long long)dt);
  if (first) {
    a.hdr->cost_key = kCostKey;
    a.hdr->cost_cells = (uint32_t)a.n_cells;
  }
}

template <typename Real, bool kHalf, int kCoul, bool kClamp, bool kDiag, int kDrain>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(kNW / 4, kNW / 4)))
void k_pair_fs(SysArgs<Real> a, int cap) {
  // home cells in the order the binning chose (longest first)
  const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
  const uint64_t c0 = __builtin_amdgcn_s_memtime();
  // workgroup b: cell order[b % n_cells], part b / n_cells (every cell's first part first)
  const int64_t cell = a.order[blockIdx.x % a.n_cells];
  const int part = (int)(blockIdx.x / a.n_cells);
  const bool last = pair_fs<Real, kHalf, kCoul, kClamp, kDiag, kDrain>(a, cap, cell, part);
  if (last && (threadIdx.x & 63) == 0) record_cost(a, cell, part, t0, c0, blockIdx.x == 0);
}

// One launch for a batch: block b is cell order[b - cum[s]] of system s.
template <bool kHalf, int kCoul, bool kClamp, bool kDiag, int kDrain>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(kNW / 4, kNW / 4)))
void k_pair_fs_batch(Batch<float> b, int cap) {
  const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
  const uint64_t c0 = __builtin_amdgcn_s_memtime();
  int64_t unit;
  const int s = b.pick(blockIdx.x, unit);
  const int64_t cell = b.sys[s].order[unit % b.sys[s].n_cells];
  const int part = (int)(unit / b.sys[s].n_cells);
  const bool last = pair_fs<float, kHalf, kCoul, kClamp, kDiag, kDrain>(b.sys[s], cap, cell, part);
  if (last && (threadIdx.x & 63) == 0) record_cost(b.sys[s], cell, part, t0, c0, unit == 0);
}

template <bool H, int S, bool C, bool D, int R>
struct launch_tag {
  static constexpr bool half = H, clamp = C, diag = D;
  static constexpr int coul = S, drain = R;
};

// Neighbour atoms staged in LDS per pass (a multiple of 64).
template <typename Real>
int fs_cap(int n_types, bool half, bool diag, int drain) {
  int cap = (kLdsBytes - lds_layout<Real>(0, n_types, half, diag, drain).total) /
            slot_bytes<Real>(half, diag);
  cap -= cap % 64;
  while (cap > 0 && lds_layout<Real>(cap, n_types, half, diag, drain).total > kLdsBytes) cap -= 64;
  return cap;
}

// The kernel instance for a system's flags: half or full shell, how the switch applies
// (whole energy with the clamp, whole energy, or LJ only), and the drain depth (other
// depths than the default only for the float32 half shell with the clamp; the API checks
// that).
template <typename Real, typename Args, typename Launch>
hipError_t dispatch(const SysArgs<Real>& a, const Args& args, int n_types, int64_t blocks,
                    hipStream_t stream, Launch launch) {
  const bool half = a.half_shell != 0;
  const bool diag = (a.flags & MD_DIAG_COUNTERS) != 0;
  const bool trunc = (a.flags & MD_COULOMB_TRUNCATED) != 0;
  const bool ewald = (a.flags & MD_COULOMB_EWALD) != 0;
  const bool clamp = !trunc && !ewald && a.inv_sw > Real(0);
  const int drain = md_pair_drain(a.flags);
  if (drain != kDrainDefault && !(half && clamp && sizeof(Real) == 4)) return hipErrorInvalidValue;
  const int cap = fs_cap<Real>(n_types, half, diag, drain);
  const size_t shmem = (size_t)lds_layout<Real>(cap, n_types, half, diag, drain).total;
  const dim3 grid((unsigned)blocks), block(kThreads);
  auto go = [&](auto h, auto d) {
    constexpr bool H = decltype(h)::value, D = decltype(d)::value;
    if (clamp) {
      if constexpr (H && sizeof(Real) == 4) {
        if (drain == 1) return launch(launch_tag<H, kCoulSwitched, true, D, 1>(), grid, block, shmem, stream, args, cap);
        if (drain == 3) return launch(launch_tag<H, kCoulSwitched, true, D, 3>(), grid, block, shmem, stream, args, cap);
        if (drain == 4) return launch(launch_tag<H, kCoulSwitched, true, D, 4>(), grid, block, shmem, stream, args, cap);
      }
      launch(launch_tag<H, kCoulSwitched, true, D, kDrainDefault>(), grid, block, shmem, stream, args, cap);
    } else if (ewald) {
      launch(launch_tag<H, kCoulEwald, false, D, kDrainDefault>(), grid, block, shmem, stream, args, cap);
    } else if (!trunc) {
      launch(launch_tag<H, kCoulSwitched, false, D, kDrainDefault>(), grid, block, shmem, stream, args, cap);
    } else {
      launch(launch_tag<H, kCoulPlain, false, D, kDrainDefault>(), grid, block, shmem, stream, args, cap);
    }
  };
  using T = std::true_type;
  using F = std::false_type;
  if (half) {
    if (diag) go(T(), T()); else go(T(), F());
  } else {
    if (diag) go(F(), T()); else go(F(), F());
  }
  return hipGetLastError();
}

}  // namespace

template <typename Real>
hipError_t launch_pair_fs(const SysArgs<Real>& a, hipStream_t stream) {
  if (a.n == 0) return hipSuccess;
  return dispatch(a, a, a.n_types, a.n_cells * a.fs_split, stream,
                  [](auto tag, dim3 g, dim3 b, size_t sh, hipStream_t st, const SysArgs<Real>& x,
                     int cap) {
                    using Tg = decltype(tag);
                    hipLaunchKernelGGL(
                        (k_pair_fs<Real, Tg::half, Tg::coul, Tg::clamp, Tg::diag, Tg::drain>), g, b,
                        sh, st, x, cap);
                  });
}

template hipError_t launch_pair_fs<float>(const SysArgs<float>&, hipStream_t);
template hipError_t launch_pair_fs<double>(const SysArgs<double>&, hipStream_t);

hipError_t launch_pair_fs_batch(const Batch<float>& b0, hipStream_t stream) {
  Batch<float> b = b0;
  int nt = 1;
  b.cum[0] = 0;
  for (int s = 0; s < b.n; ++s) {
    b.cum[s + 1] = b.cum[s] + b.sys[s].n_cells * b.sys[s].fs_split;
    nt = b.sys[s].n_types > nt ? b.sys[s].n_types : nt;
  }
  return dispatch(b.sys[0], b, nt, b.cum[b.n], stream,
                  [](auto tag, dim3 g, dim3 bl, size_t sh, hipStream_t st, const Batch<float>& x,
                     int cap) {
                    using Tg = decltype(tag);
                    hipLaunchKernelGGL(
                        (k_pair_fs_batch<Tg::half, Tg::coul, Tg::clamp, Tg::diag, Tg::drain>), g, bl,
                        sh, st, x, cap);
                  });
}

}  // namespace md
