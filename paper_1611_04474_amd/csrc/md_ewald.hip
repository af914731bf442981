// Ewald reciprocal-space sum: the Coulomb energy and forces beyond the short-range kernel.
//
// Section 2.1 splits the non-bonded work at the cutoff and hands the Coulomb part beyond
// it to an approximation outside the short-range kernel. Read here as Ewald summation of
// the periodic box: the short-range kernel (MD_COULOMB_EWALD) evaluates the screened term
// k q_i q_j erfc(alpha r)/r inside the cutoff, and this file the smooth rest,
//   E_recip = (4 pi k / V) sum_{half space of kv} w(kv) |S(kv)|^2,
//   w(kv)   = exp(-|kv|^2 / (4 alpha^2)) / |kv|^2,   S(kv) = sum_j q_j exp(i kv . r_j),
//   F_i     = q_i sum_{half space} kv Im(G(kv) exp(i kv . r_i)),  G = (8 pi k / V) w conj(S),
// over kv = 2 pi (mx/Lx, my/Ly, mz/Lz) with |m_d| <= kmax_d, one of each pair +-kv (the
// two give equal terms), plus the self term -k alpha/sqrt(pi) sum q^2 and the neutralising
// background -k pi Q^2 / (2 V alpha^2).
//
// Phases are exact modulo one turn: each atom's fractional coordinate is held as a 32-bit
// fixed-point fraction u, so m u (mod 2^32) is the phase of wave number m with no rounding,
// and only the final sine and cosine round. Wave vectors are grouped in rows (mx, my), each
// row holding every mz; the kernels are
//   k_ew_setup    per atom: fractions u, charge, NaN check, partial sums of q^2 and q;
//   k_ew_tables   per atom and wave number: exp(2 pi i m u) per axis, float2 [m][atom];
//   k_ew_sf       structure factors: a wave per row, a lane per mz, atoms of a chunk in
//                 LDS tiles of 64 (W = q X Y per (row, atom), Z per (atom, mz)); per-chunk
//                 partial sums;
//   k_ew_g        per wave vector: the chunks' partials summed in a fixed order (float64),
//                 w(kv), the energy term and G; per-row energy partials;
//   k_ew_force    a thread per atom: its Z factors in registers, per row one sine/cosine
//                 of the exact (mx, my) phase and a complex dot product of G and Z over mz;
//   k_ew_energy   one workgroup: fixed-order sum of the row energies, self and background.
// Every sum runs in a fixed order, so the results are the same bits on every run.
#include <math.h>

#include "md_common.hpp"

namespace md {
namespace {

constexpr int kEwTile = 64;       // atoms per LDS tile of the structure-factor kernel
constexpr int kEwRows = 64;       // rows per structure-factor workgroup (4 tiles of 16)
constexpr int kEwZ = 64;          // mz values per chunk of the force kernel (A operands in
                                  // registers), and the padding of G's rows
constexpr int kEwMaxK = 255;      // largest kmax per axis

struct EwArgs {
  int64_t n;
  const float* pos;               // [n][3], caller order
  const float* q;                 // [n]
  float* force;                   // [n][3]
  double* energy;                 // [1]
  int accumulate;
  WsHeader* hdr;
  uint4* ups;                     // [n]: fractions ux, uy, uz and the charge's bits
  float2* tab;                    // [(kx+1) + (2ky+1) + (2kz+1)][n]: X, then Y, then Z
  float2* parts;                  // [chunks][R][nzc] partial structure factors
  float2* g;                      // [R][nzc_pad] G (zero where excluded and in the padding)
  double* erow;                   // [R][zblocks] energy partials
  double2* qpart;                 // [qblocks] (sum q^2, sum q) per setup block
  int kx, ky, kz, nzc, nzc_pad, zblocks;
  int64_t rows, chunks, chunk_atoms, qblocks;
  double L[3];
  double alpha, coulomb_k;
};

__host__ __device__ inline int64_t ew_rows(int kx, int ky) {
  return (int64_t)kx * (2 * ky + 1) + (ky + 1);
}

// Row r -> (mx, my): rows 0..ky are (0, my >= 0), then mx >= 1 with every my.
__device__ inline void ew_row(const EwArgs& a, int64_t r, int& mx, int& my) {
  if (r <= a.ky) {
    mx = 0;
    my = (int)r;
  } else {
    const int64_t s = r - (a.ky + 1);
    mx = 1 + (int)(s / (2 * a.ky + 1));
    my = (int)(s % (2 * a.ky + 1)) - a.ky;
  }
}

// exp(2 pi i m u / 2^32) for the phase m u taken modulo 2^32 (exact), as (cos, sin).
__device__ inline float2 ew_phase(uint32_t ph) {
  float s, c;
  sincospif((float)(int32_t)ph * 4.656612873077393e-10f, &s, &c);   // 2^-31: units of pi
  return make_float2(c, s);
}

__global__ __launch_bounds__(256) void k_ew_setup(EwArgs a) {
  __shared__ double sq2[256], sq[256];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double q2 = 0.0, q1 = 0.0;
  if (i < a.n) {
    uint32_t st = 0, u[3];
    for (int d = 0; d < 3; ++d) {
      const double x = (double)a.pos[3 * i + d];
      if (x != x) {
        st |= MD_STATUS_NAN;
        u[d] = 0;
        continue;
      }
      const double s = x / a.L[d];
      const double f = s - floor(s);                               // [0, 1)
      u[d] = (uint32_t)(unsigned long long)llrint(f * 4294967296.0);   // 2^32 wraps to 0
    }
    const float qi = a.q[i];
    if (qi != qi) st |= MD_STATUS_NAN;
    a.ups[i] = make_uint4(u[0], u[1], u[2], __float_as_uint(qi));
    q2 = (double)qi * (double)qi;
    q1 = (double)qi;
    if (st) atomicOr(&a.hdr->status, st);
  }
  sq2[threadIdx.x] = q2;
  sq[threadIdx.x] = q1;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      sq2[threadIdx.x] += sq2[threadIdx.x + off];
      sq[threadIdx.x] += sq[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) a.qpart[blockIdx.x] = make_double2(sq2[0], sq[0]);
}

// Table row t: X (mx = 0..kx), Y (my = -ky..ky), Z (mz = -kz..kz), each [m][atom].
__global__ __launch_bounds__(256) void k_ew_tables(EwArgs a) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= a.n) return;
  const int t = blockIdx.y;
  const uint4 u = a.ups[i];
  int m;
  uint32_t ua;
  if (t <= a.kx) {
    m = t;
    ua = u.x;
  } else if (t <= a.kx + 2 * a.ky + 1) {
    m = t - (a.kx + 1) - a.ky;
    ua = u.y;
  } else {
    m = t - (a.kx + 2 * a.ky + 2) - a.kz;
    ua = u.z;
  }
  a.tab[(int64_t)t * a.n + i] = ew_phase((uint32_t)m * ua);
}

// Structure factors as a complex matrix product over atoms, on the matrix cores:
// S[r][mz] = sum_j W[r][j] Z[j][mz], W = q X[mx(r)] Y[my(r)]. A workgroup takes 64 rows x
// 64 values of mz x one chunk of atoms; wave w owns the 16 x 16 output tile (rows
// 16 (w / 4) .., mz 16 (w % 4) ..). Per tile of 64 atoms the workgroup writes W (computed)
// and Z (loaded) to LDS, atom-major and padded so that both the transposing stores and the
// operand reads spread over the banks; each wave then runs 16 steps of 4 atoms, each step
// four v_mfma_f32_16x16x4f32 (re re, -im im, re im, im re). In a 16x16x4 f32 product, lane
// l supplies A[l % 16][l / 16] and B[l / 16][l % 16] and holds D[4 (l / 16) + i][l % 16],
// i = 0..3. The accumulation order is fixed, so the partial sums are the same bits on every
// run.
typedef float ew_v4f __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_ew_sf(EwArgs a) {
  __shared__ float2 sW[kEwTile][kEwRows + 1];   // [atom][row]
  __shared__ float2 sZ[kEwTile][64 + 1];        // [atom][mz]
  const int t = threadIdx.x;
  const int w = t >> 6, lane = t & 63;
  const int64_t r0 = (int64_t)blockIdx.x * kEwRows;
  const int z0 = blockIdx.z * 64;
  const int64_t a0 = (int64_t)blockIdx.y * a.chunk_atoms;
  const int64_t a1 = a0 + a.chunk_atoms < a.n ? a0 + a.chunk_atoms : a.n;
  // staging roles: atom ta = t % 64 of the tile; W for rows 4 (t / 64) .. + 3, Z for mz
  // t / 64 + 16 p (p = 0..3)
  const int ta = t & 63, tg = t >> 6;
  int mxs[4], mys[4];
  bool rok[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t r = r0 + 4 * tg + k;
    rok[k] = r < a.rows;
    mxs[k] = 0;
    mys[k] = 0;
    if (rok[k]) ew_row(a, r, mxs[k], mys[k]);
  }
  const float2* Z = a.tab + (int64_t)(a.kx + 2 * a.ky + 2) * a.n;
  // this wave's output tile and its operand columns
  const int rt = w >> 2, zt = w & 3;
  const int ar = 16 * rt + (lane & 15);   // A row (this lane's row of W)
  const int bz = 16 * zt + (lane & 15);   // B column (this lane's mz)
  const int kk = lane >> 4;               // this lane's atom within a step
  ew_v4f dre = {0.f, 0.f, 0.f, 0.f}, dim = {0.f, 0.f, 0.f, 0.f};
  // this thread's staging values of one tile, loaded a tile ahead of their use
  float2 wn[4], zn[4];
  auto load_tile = [&](int64_t t0) __attribute__((always_inline)) {
    const int64_t j = t0 + ta;
    const bool jok = j < a1;
    const float qj = jok ? __uint_as_float(a.ups[j].w) : 0.f;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      float2 wv = make_float2(0.f, 0.f);
      if (jok && rok[k]) {
        const float2 x = a.tab[(int64_t)mxs[k] * a.n + j];
        const float2 y = a.tab[(int64_t)(a.kx + 1 + mys[k] + a.ky) * a.n + j];
        wv = make_float2(qj * (x.x * y.x - x.y * y.y), qj * (x.x * y.y + x.y * y.x));
      }
      wn[k] = wv;
    }
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const int zi = z0 + tg + 16 * p;
      zn[p] = (jok && zi < a.nzc) ? Z[(int64_t)zi * a.n + j] : make_float2(0.f, 0.f);
    }
  };
  if (a0 < a1) load_tile(a0);
  for (int64_t t0 = a0; t0 < a1; t0 += kEwTile) {
#pragma unroll
    for (int k = 0; k < 4; ++k) sW[ta][4 * tg + k] = wn[k];
#pragma unroll
    for (int p = 0; p < 4; ++p) sZ[ta][tg + 16 * p] = zn[p];
    __syncthreads();
    if (t0 + kEwTile < a1) load_tile(t0 + kEwTile);
    // atoms past the chunk's end hold W = Z = 0, so every step can run in full
#pragma unroll 4
    for (int s = 0; s < kEwTile / 4; ++s) {
      const float2 av = sW[4 * s + kk][ar];
      const float2 bv = sZ[4 * s + kk][bz];
      dre = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, bv.x, dre, 0, 0, 0);
      dre = __builtin_amdgcn_mfma_f32_16x16x4f32(-av.y, bv.y, dre, 0, 0, 0);
      dim = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, bv.y, dim, 0, 0, 0);
      dim = __builtin_amdgcn_mfma_f32_16x16x4f32(av.y, bv.x, dim, 0, 0, 0);
    }
    __syncthreads();
  }
  const int zi = z0 + bz;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t r = r0 + 16 * rt + 4 * kk + i;
    if (r < a.rows && zi < a.nzc)
      a.parts[((int64_t)blockIdx.y * a.rows + r) * a.nzc + zi] = make_float2(dre[i], dim[i]);
  }
}

// Per wave vector: S from the chunks (fixed order, float64), the energy term and G.
__global__ __launch_bounds__(64) void k_ew_g(EwArgs a) {
  __shared__ double se[64];
  const int64_t r = blockIdx.x;
  const int zi = blockIdx.y * 64 + threadIdx.x;
  int mx, my;
  ew_row(a, r, mx, my);
  double e = 0.0;
  float2 gv = make_float2(0.f, 0.f);
  if (zi < a.nzc) {
    const int mz = zi - a.kz;
    const bool use = mx > 0 || my > 0 || mz > 0;   // half space, kv != 0
    if (use) {
      double sr = 0.0, si = 0.0;
      for (int64_t c = 0; c < a.chunks; ++c) {
        const float2 p = a.parts[(c * a.rows + r) * a.nzc + zi];
        sr += (double)p.x;
        si += (double)p.y;
      }
      const double pi = 3.141592653589793;
      const double kx = 2.0 * pi * mx / a.L[0], ky = 2.0 * pi * my / a.L[1],
                   kz = 2.0 * pi * mz / a.L[2];
      const double k2 = kx * kx + ky * ky + kz * kz;
      const double wk = exp(-k2 / (4.0 * a.alpha * a.alpha)) / k2;
      const double V = a.L[0] * a.L[1] * a.L[2];
      e = 4.0 * pi * a.coulomb_k / V * wk * (sr * sr + si * si);
      const double gs = 8.0 * pi * a.coulomb_k / V * wk;
      gv = make_float2((float)(gs * sr), (float)(-gs * si));   // (8 pi k / V) w conj(S)
    }
  }
  if (zi < a.nzc_pad) a.g[r * a.nzc_pad + zi] = gv;
  se[threadIdx.x] = e;
  __syncthreads();
  for (int off = 32; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) se[threadIdx.x] += se[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.erow[r * a.zblocks + blockIdx.y] = se[0];
}

// Forces as complex matrix products over mz, on the matrix cores: for atoms i and rows
// (mx, my), T[i][r] = sum_mz Z[mz][i] G[r][mz] and U[i][r] = sum_mz mz Z[mz][i] G[r][mz];
// then F_i = q_i sum_r (kx, ky) Im(xy T) + (0, 0, kz) Im(xy U) with xy = exp(i (kx x + ky
// y)) from the exact phase of (mx, my). A workgroup of 4 waves takes 64 atoms, a wave 16 of
// them (rows of A, Z of its atoms for 64 values of mz in registers) against tiles of 16
// rows of G (columns of B) staged in LDS; each step of 4 values of mz runs eight
// v_mfma_f32_16x16x4f32 (T and U, re and im parts). A lane then holds 4 atoms x 1 row of T
// and U: it adds that row's force terms for its 4 atoms in float32 and each tile's sums into
// float64; the 16 lanes of a row group finally add their sums in a fixed butterfly.
__global__ __launch_bounds__(256) void k_ew_force(EwArgs a) {
  __shared__ float2 sG[16][kEwZ + 1];   // [row][mz] of the current tile and mz chunk
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const int kk = lane >> 4, col = lane & 15;
  const int64_t ia = (int64_t)blockIdx.x * 64 + 16 * w + col;   // this lane's A row (atom)
  const bool aok = ia < a.n;
  // the 4 atoms of this lane's D rows: 16 w + 4 kk + i
  uint32_t ux[4], uy[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t id = (int64_t)blockIdx.x * 64 + 16 * w + 4 * kk + i;
    const uint4 u = id < a.n ? a.ups[id] : make_uint4(0, 0, 0, 0);
    ux[i] = u.x;
    uy[i] = u.y;
  }
  const double pi = 3.141592653589793;
  const float kxs = (float)(2.0 * pi / a.L[0]), kys = (float)(2.0 * pi / a.L[1]),
              kzs = (float)(2.0 * pi / a.L[2]);
  double F[4][3] = {};
  const float2* Zt = a.tab + (int64_t)(a.kx + 2 * a.ky + 2) * a.n;
  for (int zc = 0; zc < a.nzc_pad; zc += kEwZ) {
    // A operands for this mz chunk: step s holds Z[zc + 4 s + kk][ia]; ns steps cover the
    // chunk's mz values below nzc
    const int ns = (min(kEwZ, a.nzc - zc) + 3) / 4;
    float2 z[kEwZ / 4];
#pragma unroll
    for (int s = 0; s < kEwZ / 4; ++s) {
      const int zi = zc + 4 * s + kk;
      z[s] = (aok && zi < a.nzc) ? Zt[(int64_t)zi * a.n + ia] : make_float2(0.f, 0.f);
    }
    for (int64_t r0 = 0; r0 < a.rows; r0 += 16) {
      __syncthreads();
      for (int e = t; e < 16 * kEwZ; e += 256) {
        const int rr = e / kEwZ, k = e % kEwZ;
        sG[rr][k] = r0 + rr < a.rows ? a.g[(r0 + rr) * a.nzc_pad + zc + k] : make_float2(0.f, 0.f);
      }
      __syncthreads();
      ew_v4f tre = {0.f, 0.f, 0.f, 0.f}, tim = tre, ure = tre, uim = tre;
#pragma unroll
      for (int s = 0; s < kEwZ / 4; ++s) {
        if (s < ns) {   // steps past the chunk's last mz are skipped (uniform)
          const float2 g = sG[col][4 * s + kk];
          const float mz = (float)(zc + 4 * s + kk - a.kz);
          const float2 gm = make_float2(mz * g.x, mz * g.y);
          tre = __builtin_amdgcn_mfma_f32_16x16x4f32(z[s].x, g.x, tre, 0, 0, 0);
          tre = __builtin_amdgcn_mfma_f32_16x16x4f32(-z[s].y, g.y, tre, 0, 0, 0);
          tim = __builtin_amdgcn_mfma_f32_16x16x4f32(z[s].x, g.y, tim, 0, 0, 0);
          tim = __builtin_amdgcn_mfma_f32_16x16x4f32(z[s].y, g.x, tim, 0, 0, 0);
          ure = __builtin_amdgcn_mfma_f32_16x16x4f32(z[s].x, gm.x, ure, 0, 0, 0);
          ure = __builtin_amdgcn_mfma_f32_16x16x4f32(-z[s].y, gm.y, ure, 0, 0, 0);
          uim = __builtin_amdgcn_mfma_f32_16x16x4f32(z[s].x, gm.y, uim, 0, 0, 0);
          uim = __builtin_amdgcn_mfma_f32_16x16x4f32(z[s].y, gm.x, uim, 0, 0, 0);
        }
      }
      // this lane's row r0 + col against its 4 atoms (rows past the end hold T = U = 0)
      const int64_t r = r0 + col;
      int mx = 0, my = 0;
      if (r < a.rows) ew_row(a, r, mx, my);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float2 xy = ew_phase((uint32_t)mx * ux[i] + (uint32_t)my * uy[i]);
        const float imt = fmaf(xy.x, tim[i], xy.y * tre[i]);   // Im(xy T)
        const float imu = fmaf(xy.x, uim[i], xy.y * ure[i]);   // Im(xy U)
        F[i][0] += (double)((float)mx * kxs * imt);
        F[i][1] += (double)((float)my * kys * imt);
        F[i][2] += (double)(kzs * imu);
      }
    }
  }
  // sum over the 16 lanes of each row group (fixed butterfly), then lane 16 kk + 0 writes
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
      for (int sft = 1; sft < 16; sft <<= 1) F[i][d] += __shfl_xor(F[i][d], sft);
  if (col == 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t id = (int64_t)blockIdx.x * 64 + 16 * w + 4 * kk + i;
      if (id >= a.n) continue;
      const float qi = __uint_as_float(a.ups[id].w);
      float* out = a.force + 3 * id;
      for (int d = 0; d < 3; ++d) {
        const float v = (float)((double)qi * F[i][d]);
        out[d] = a.accumulate ? out[d] + v : v;
      }
    }
  }
}

// Energy: row partials, then self and background terms, in a fixed order.
__global__ __launch_bounds__(256) void k_ew_energy(EwArgs a) {
  __shared__ double s[256], s2[256], s1[256];
  double e = 0.0, q2 = 0.0, q1 = 0.0;
  const int64_t ne = a.rows * a.zblocks;
  for (int64_t t = threadIdx.x; t < ne; t += 256) e += a.erow[t];
  for (int64_t t = threadIdx.x; t < a.qblocks; t += 256) {
    q2 += a.qpart[t].x;
    q1 += a.qpart[t].y;
  }
  s[threadIdx.x] = e;
  s2[threadIdx.x] = q2;
  s1[threadIdx.x] = q1;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      s[threadIdx.x] += s[threadIdx.x + off];
      s2[threadIdx.x] += s2[threadIdx.x + off];
      s1[threadIdx.x] += s1[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double pi = 3.141592653589793;
    const double V = a.L[0] * a.L[1] * a.L[2];
    const double self = -a.coulomb_k * a.alpha / sqrt(pi) * s2[0];
    const double bg = -a.coulomb_k * pi * s1[0] * s1[0] / (2.0 * V * a.alpha * a.alpha);
    *a.energy = s[0] + self + bg;
  }
}

__global__ void k_ew_clear_status(WsHeader* hdr) { hdr->status = 0; }

struct EwPlan {
  int kx, ky, kz, nzc, nzc_pad, zblocks;
  int64_t rows, chunks, chunk_atoms, qblocks;
  size_t off_ups, off_tab, off_parts, off_g, off_erow, off_qpart, total;
};

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

md_status ew_plan(const md_params* p, int64_t n, const int32_t kmax[3], EwPlan* pl) {
  if (!p || !kmax || n < 0 || n > kMaxAtoms) return MD_ERR_INVALID_ARG;
  if (!(p->ewald_alpha > 0) || !isfinite(p->ewald_alpha) || !isfinite(p->coulomb_k))
    return MD_ERR_INVALID_ARG;
  for (int d = 0; d < 3; ++d) {
    if (!(p->box[d] > 0) || !isfinite(p->box[d])) return MD_ERR_INVALID_ARG;
    if (kmax[d] < 0 || kmax[d] > kEwMaxK) return MD_ERR_INVALID_ARG;
  }
  if (kmax[0] + kmax[1] + kmax[2] == 0) return MD_ERR_INVALID_ARG;
  pl->kx = kmax[0];
  pl->ky = kmax[1];
  pl->kz = kmax[2];
  pl->nzc = 2 * pl->kz + 1;
  pl->nzc_pad = (pl->nzc + kEwZ - 1) / kEwZ * kEwZ;
  pl->zblocks = (pl->nzc_pad + 63) / 64;   // covers the padding of G, which k_ew_g zeroes
  pl->rows = ew_rows(pl->kx, pl->ky);
  // atom chunks: enough workgroups to fill the chip, chunks of whole tiles
  const int64_t rb = (pl->rows + kEwRows - 1) / kEwRows;
  const int64_t tiles = (n + kEwTile - 1) / kEwTile > 0 ? (n + kEwTile - 1) / kEwTile : 1;
  int64_t chunks = (512 + rb * pl->zblocks - 1) / (rb * pl->zblocks);   // two per compute unit
  chunks = chunks < 1 ? 1 : chunks > tiles ? tiles : chunks;
  pl->chunk_atoms = (tiles + chunks - 1) / chunks * kEwTile;
  pl->chunks = n > 0 ? (n + pl->chunk_atoms - 1) / pl->chunk_atoms : 1;
  pl->qblocks = (n + 255) / 256 > 0 ? (n + 255) / 256 : 1;
  const size_t nn = (size_t)(n > 0 ? n : 1);
  const int64_t trows = (pl->kx + 1) + (2 * pl->ky + 1) + pl->nzc;
  size_t o = a256(sizeof(WsHeader));
  pl->off_ups = o;   o = a256(o + sizeof(uint4) * nn);
  pl->off_tab = o;   o = a256(o + sizeof(float2) * (size_t)trows * nn);
  pl->off_parts = o; o = a256(o + sizeof(float2) * (size_t)pl->chunks * pl->rows * pl->nzc);
  pl->off_g = o;     o = a256(o + sizeof(float2) * (size_t)pl->rows * pl->nzc_pad);
  pl->off_erow = o;  o = a256(o + sizeof(double) * (size_t)pl->rows * pl->zblocks);
  pl->off_qpart = o; o = a256(o + sizeof(double2) * (size_t)pl->qblocks);
  pl->total = o;
  return MD_OK;
}

}  // namespace
}  // namespace md

extern "C" {

size_t md_ewald_workspace_bytes(const md_params* p, int64_t n_atoms, const int32_t kmax[3]) {
  md::EwPlan pl;
  return md::ew_plan(p, n_atoms, kmax, &pl) == MD_OK ? pl.total : 0;
}

md_status md_ewald_recip_f32(const md_params* p, int64_t n_atoms, const float* d_pos,
                             const float* d_charge, const int32_t kmax[3], float* d_force,
                             double* d_energy, int32_t accumulate, void* d_ws, size_t ws_bytes,
                             void* stream) {
  md::EwPlan pl;
  md_status s = md::ew_plan(p, n_atoms, kmax, &pl);
  if (s != MD_OK) return s;
  if (!d_energy || ((uintptr_t)d_energy & 7)) return MD_ERR_INVALID_ARG;
  if (n_atoms > 0 && (!d_pos || !d_charge || !d_force ||
                      (((uintptr_t)d_pos | (uintptr_t)d_charge | (uintptr_t)d_force) & 3)))
    return MD_ERR_INVALID_ARG;
  if (!d_ws || ((uintptr_t)d_ws & 255) || ws_bytes < pl.total) return MD_ERR_WORKSPACE;
  md::EwArgs a;
  char* b = (char*)d_ws;
  a.n = n_atoms;
  a.pos = d_pos;
  a.q = d_charge;
  a.force = d_force;
  a.energy = d_energy;
  a.accumulate = accumulate ? 1 : 0;
  a.hdr = (md::WsHeader*)b;
  a.ups = (uint4*)(b + pl.off_ups);
  a.tab = (float2*)(b + pl.off_tab);
  a.parts = (float2*)(b + pl.off_parts);
  a.g = (float2*)(b + pl.off_g);
  a.erow = (double*)(b + pl.off_erow);
  a.qpart = (double2*)(b + pl.off_qpart);
  a.kx = pl.kx;
  a.ky = pl.ky;
  a.kz = pl.kz;
  a.nzc = pl.nzc;
  a.nzc_pad = pl.nzc_pad;
  a.zblocks = pl.zblocks;
  a.rows = pl.rows;
  a.chunks = pl.chunks;
  a.chunk_atoms = pl.chunk_atoms;
  a.qblocks = pl.qblocks;
  for (int d = 0; d < 3; ++d) a.L[d] = (double)(float)p->box[d];   // the float32 box
  a.alpha = p->ewald_alpha;
  a.coulomb_k = p->coulomb_k;
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(md::k_ew_clear_status, dim3(1), dim3(1), 0, st, a.hdr);
  if (n_atoms > 0) {
    const unsigned nb = (unsigned)((n_atoms + 255) / 256);
    const unsigned trows = (unsigned)((pl.kx + 1) + (2 * pl.ky + 1) + pl.nzc);
    hipLaunchKernelGGL(md::k_ew_setup, dim3(nb), dim3(256), 0, st, a);
    hipLaunchKernelGGL(md::k_ew_tables, dim3(nb, trows), dim3(256), 0, st, a);
    hipLaunchKernelGGL(md::k_ew_sf,
                       dim3((unsigned)((pl.rows + md::kEwRows - 1) / md::kEwRows),
                            (unsigned)pl.chunks, (unsigned)pl.zblocks),
                       dim3(1024), 0, st, a);
    hipLaunchKernelGGL(md::k_ew_g, dim3((unsigned)pl.rows, (unsigned)pl.zblocks), dim3(64), 0, st, a);
    hipLaunchKernelGGL(md::k_ew_force, dim3((unsigned)((n_atoms + 63) / 64)), dim3(256), 0, st, a);
  } else {
    // no atoms: every term is zero
    a.qblocks = 0;
    a.rows = 0;
  }
  hipLaunchKernelGGL(md::k_ew_energy, dim3(1), dim3(256), 0, st, a);
  return hipGetLastError() == hipSuccess ? MD_OK : MD_ERR_HIP;
}

}  // extern "C"
