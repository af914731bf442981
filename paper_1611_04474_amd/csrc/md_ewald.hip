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
constexpr int kEwRows = 16;       // rows per structure-factor workgroup (one per wave)
constexpr int kEwZ = 32;          // mz values held in registers by the force kernel
constexpr int kEwForceRows = 16;  // rows of G staged in LDS at a time by the force kernel
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

// Structure factors: workgroup = kEwRows rows x 64 values of mz x one chunk of atoms.
__global__ __launch_bounds__(1024) void k_ew_sf(EwArgs a) {
  __shared__ float2 sW[kEwRows][kEwTile];
  __shared__ float2 sZ[kEwTile][65];   // padded: the transposing stores spread over banks
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * kEwRows + w;
  const int z0 = blockIdx.z * 64;
  const int64_t a0 = (int64_t)blockIdx.y * a.chunk_atoms;
  const int64_t a1 = a0 + a.chunk_atoms < a.n ? a0 + a.chunk_atoms : a.n;
  int mx = 0, my = 0;
  if (r < a.rows) ew_row(a, r, mx, my);
  const float2* X = a.tab + (int64_t)mx * a.n;
  const float2* Y = a.tab + (int64_t)(a.kx + 1 + my + a.ky) * a.n;
  const float2* Z = a.tab + (int64_t)(a.kx + 2 * a.ky + 2) * a.n;
  float sr = 0.f, si = 0.f;
  for (int64_t t0 = a0; t0 < a1; t0 += kEwTile) {
    {
      // W = q X[mx] Y[my] of atom t0 + lane for this wave's row
      const int64_t j = t0 + lane;
      float2 wv = make_float2(0.f, 0.f);
      if (j < a1 && r < a.rows) {
        const float qj = __uint_as_float(a.ups[j].w);
        const float2 x = X[j], y = Y[j];
        wv = make_float2(qj * (x.x * y.x - x.y * y.y), qj * (x.x * y.y + x.y * y.x));
      }
      sW[w][lane] = wv;
    }
    // Z of the tile's atoms for mz = z0 .. z0 + 63: thread (k, aa) loads rows k, k + 16, ..
    for (int zz = w; zz < 64; zz += kEwRows) {
      const int64_t j = t0 + lane;
      const int zi = z0 + zz;
      sZ[lane][zz] = (j < a1 && zi < a.nzc) ? Z[(int64_t)zi * a.n + j] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    const int na = (int)(a1 - t0 < kEwTile ? a1 - t0 : kEwTile);
    for (int aa = 0; aa < na; ++aa) {
      const float2 wv = sW[w][aa];
      const float2 zv = sZ[aa][lane];
      sr = fmaf(wv.x, zv.x, sr);
      sr = fmaf(-wv.y, zv.y, sr);
      si = fmaf(wv.x, zv.y, si);
      si = fmaf(wv.y, zv.x, si);
    }
    __syncthreads();
  }
  const int zi = z0 + lane;
  if (r < a.rows && zi < a.nzc)
    a.parts[((int64_t)blockIdx.y * a.rows + r) * a.nzc + zi] = make_float2(sr, si);
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

// Forces: a thread per atom, kEwZ values of mz at a time in registers.
__global__ __launch_bounds__(256) void k_ew_force(EwArgs a) {
  __shared__ float2 sG[kEwForceRows][kEwZ];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool live = i < a.n;
  const uint4 u = live ? a.ups[i] : make_uint4(0, 0, 0, 0);
  const float qi = __uint_as_float(u.w);
  const double pi = 3.141592653589793;
  const float kxs = (float)(2.0 * pi / a.L[0]), kys = (float)(2.0 * pi / a.L[1]),
              kzs = (float)(2.0 * pi / a.L[2]);
  double F[3] = {0.0, 0.0, 0.0};
  for (int zc = 0; zc < a.nzc_pad; zc += kEwZ) {
    float2 z[kEwZ];
    const float2* Z = a.tab + (int64_t)(a.kx + 2 * a.ky + 2 + zc) * a.n;
#pragma unroll
    for (int k = 0; k < kEwZ; ++k)
      z[k] = (live && zc + k < a.nzc) ? Z[(int64_t)k * a.n + i] : make_float2(0.f, 0.f);
    for (int64_t r0 = 0; r0 < a.rows; r0 += kEwForceRows) {
      __syncthreads();
      for (int e = threadIdx.x; e < kEwForceRows * kEwZ; e += 256) {
        const int rr = e / kEwZ, k = e % kEwZ;
        sG[rr][k] = (r0 + rr < a.rows) ? a.g[(r0 + rr) * a.nzc_pad + zc + k] : make_float2(0.f, 0.f);
      }
      __syncthreads();
      float fx = 0.f, fy = 0.f, fz = 0.f;
      const int nr = (int)(a.rows - r0 < kEwForceRows ? a.rows - r0 : kEwForceRows);
      for (int rr = 0; rr < nr; ++rr) {
        int mx, my;
        ew_row(a, r0 + rr, mx, my);
        // U = sum G Z, V = sum mz G Z over this chunk of mz
        float ur = 0.f, ui = 0.f, vr = 0.f, vi = 0.f;
#pragma unroll
        for (int k = 0; k < kEwZ; ++k) {
          const float2 gv = sG[rr][k];
          const float pr = fmaf(gv.x, z[k].x, -gv.y * z[k].y);
          const float pim = fmaf(gv.x, z[k].y, gv.y * z[k].x);
          const float mz = (float)(zc + k - a.kz);
          ur += pr;
          ui += pim;
          vr = fmaf(mz, pr, vr);
          vi = fmaf(mz, pim, vi);
        }
        // exp(i (kx x + ky y)) from the exact phase of (mx, my)
        const float2 xy = ew_phase((uint32_t)mx * u.x + (uint32_t)my * u.y);
        const float imu = fmaf(xy.x, ui, xy.y * ur);    // Im(xy U)
        const float imv = fmaf(xy.x, vi, xy.y * vr);    // Im(xy V)
        fx = fmaf((float)mx * kxs, imu, fx);
        fy = fmaf((float)my * kys, imu, fy);
        fz = fmaf(kzs, imv, fz);
      }
      F[0] += (double)fx;
      F[1] += (double)fy;
      F[2] += (double)fz;
    }
  }
  if (!live) return;
  float* out = a.force + 3 * i;
  for (int d = 0; d < 3; ++d) {
    const float v = (float)((double)qi * F[d]);
    out[d] = a.accumulate ? out[d] + v : v;
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
  int64_t chunks = (2048 + rb * pl->zblocks - 1) / (rb * pl->zblocks);
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
    hipLaunchKernelGGL(md::k_ew_force, dim3(nb), dim3(256), 0, st, a);
  } else {
    // no atoms: every term is zero
    a.qblocks = 0;
    a.rows = 0;
  }
  hipLaunchKernelGGL(md::k_ew_energy, dim3(1), dim3(256), 0, st, a);
  return hipGetLastError() == hipSuccess ? MD_OK : MD_ERR_HIP;
}

}  // extern "C"
