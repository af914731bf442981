// C ABI entry points: argument checks, the cell grid, the workspace carve-up, and
// the launch sequence binning -> pair -> finalize on the caller's stream.
#include <math.h>
#include <string.h>

#include <atomic>
#include <mutex>

#include "md_common.hpp"

namespace md {

// Workspace of md_forces_f32_noalloc: one per device, held from the library's first use
// on that device until the process ends. Host code reaches it only through the device
// address that hipGetSymbolAddress returns for the current device (noalloc_scratch).
constexpr size_t kScratchBytes = (size_t)MD_NOALLOC_MAX_WORKSPACE_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::atomic<void*> g_scratch[kMaxDevices];
static std::mutex g_scratch_mu;

// Device address of the current device's scratch array, looked up once per device.
static md_status noalloc_scratch(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return MD_ERR_HIP;
  if (dev < 0 || dev >= kMaxDevices) return MD_ERR_CAPACITY;
  void* ptr = g_scratch[dev].load(std::memory_order_acquire);
  if (!ptr) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    ptr = g_scratch[dev].load(std::memory_order_relaxed);
    if (!ptr) {
      if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
        return MD_ERR_HIP;
      g_scratch[dev].store(ptr, std::memory_order_release);
    }
  }
  *out = ptr;
  return MD_OK;
}

// Copies the status word of a workspace to caller memory, in stream order.
__global__ void k_copy_status(const WsHeader* hdr, uint32_t* out) { *out = hdr->status; }

static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

static md_status check_params(const md_params* p) {
  if (!p) return MD_ERR_INVALID_ARG;
  if (p->n_types < 1) return MD_ERR_INVALID_ARG;
  if (p->n_types > kMaxTypes) return MD_ERR_CAPACITY;
  if (!p->sigma || !p->epsilon) return MD_ERR_INVALID_ARG;
  for (int t = 0; t < p->n_types; ++t) {
    if (!isfinite(p->sigma[t]) || !isfinite(p->epsilon[t]) || p->epsilon[t] < 0)
      return MD_ERR_INVALID_ARG;
  }
  if (!(p->r_cut > 0) || !isfinite(p->r_cut)) return MD_ERR_INVALID_ARG;
  if (!(p->r_switch > 0) || p->r_switch > p->r_cut) return MD_ERR_INVALID_ARG;
  if (!isfinite(p->coulomb_k)) return MD_ERR_INVALID_ARG;
  const uint32_t known = MD_ACCUM_F32_ATOMIC | MD_COULOMB_TRUNCATED | MD_DIAG_COUNTERS |
                         MD_PAIR_PREDICATED | MD_PAIR_FULL_SHELL | MD_PAIR_DRAIN_MASK |
                         MD_COULOMB_EWALD | MD_PAIR_SPLIT_MASK;
  if (p->flags & ~known) return MD_ERR_INVALID_ARG;
  // Ewald's real-space term: a finite positive splitting parameter, on the compacted kernel
  // (float32 sums only there), not together with the truncated form
  if (p->flags & MD_COULOMB_EWALD) {
    if (!(p->ewald_alpha > 0) || !isfinite(p->ewald_alpha)) return MD_ERR_INVALID_ARG;
    if (p->flags & (MD_COULOMB_TRUNCATED | MD_PAIR_PREDICATED)) return MD_ERR_INVALID_ARG;
  }
  // a work split only for the compacted kernel
  if ((p->flags & MD_PAIR_SPLIT_MASK) && (p->flags & MD_PAIR_PREDICATED)) return MD_ERR_INVALID_ARG;
  // another drain depth only for the kernel that has it: the compacted half shell with the
  // whole energy switched (the float64 path is checked in check_call)
  if ((p->flags & MD_PAIR_DRAIN_MASK) &&
      ((p->flags & (MD_ACCUM_F32_ATOMIC | MD_COULOMB_TRUNCATED | MD_PAIR_PREDICATED |
                    MD_PAIR_FULL_SHELL | MD_COULOMB_EWALD)) ||
       !(p->r_switch < p->r_cut)))
    return MD_ERR_INVALID_ARG;
  for (int d = 0; d < 3; ++d)
    if (!isfinite(p->box[d]) || !(p->box[d] > 0)) return MD_ERR_INVALID_ARG;
  return MD_OK;
}

// The compacted pair kernel serves every call except MD_PAIR_PREDICATED and float64 with
// float32 atomics, which take the predicated kernel.
static bool uses_compact(const md_params* p, int real_bytes) {
  return !(p->flags & MD_PAIR_PREDICATED) &&
         !(real_bytes == 8 && (p->flags & MD_ACCUM_F32_ATOMIC));
}

// Grid rule: n_d = floor(L_d / r_cut), one cell fewer when L_d/n_d exceeds r_cut by
// less than 1e-3 A (so rounding of a coordinate at a cell face never hides a pair),
// and at least 2 cells per axis (L >= 2 r_cut keeps the minimum image unique).
md_status make_plan(const md_params* p, int64_t n, int real_bytes, Plan* pl) {
  md_status s = check_params(p);
  if (s != MD_OK) return s;
  if (n < 0) return MD_ERR_INVALID_ARG;
  if (n > kMaxAtoms) return MD_ERR_CAPACITY;
  int64_t cells = 1;
  for (int d = 0; d < 3; ++d) {
    double L = real_bytes == 4 ? (double)(float)p->box[d] : p->box[d];
    double q = floor(L / p->r_cut);
    if (q > 1e7) return MD_ERR_CAPACITY;
    int nd = (int)q;
    if (nd >= 1 && L / nd - p->r_cut < 1e-3) nd -= 1;
    if (nd < 2) return MD_ERR_BOX_TOO_SMALL;
    pl->dims[d] = nd;
    cells *= nd;
    if (cells > kMaxCells) return MD_ERR_CAPACITY;
  }
  pl->n_cells = cells;
  pl->n_tasks = cells * kTasksPerCell;
  pl->n = n;
  pl->real_bytes = real_bytes;
  const size_t nn = (size_t)(n > 0 ? n : 1);
  size_t o = align_up(sizeof(WsHeader));
  pl->off_count = o;     o = align_up(o + sizeof(int32_t) * cells);
  pl->off_start = o;     o = align_up(o + sizeof(int32_t) * (cells + 1));
  pl->off_cell = o;      o = align_up(o + sizeof(int32_t) * nn);
  pl->off_rank = o;      o = align_up(o + sizeof(int32_t) * nn);
  const bool compact = uses_compact(p, real_bytes);
  pl->off_pos = o;       o = align_up(o + (size_t)4 * real_bytes * nn);
  pl->off_hpre = o;      o = align_up(o + (compact ? (size_t)8 * real_bytes * nn : 0));
  pl->off_type = o;      o = align_up(o + sizeof(int32_t) * nn);
  pl->off_perm = o;      o = align_up(o + sizeof(int32_t) * nn);
  // per-atom partials: 27 slots x 3 components for the predicated kernel, or three
  // 64-bit fixed-point sums (float32) or three two-word ones (float64) for the compacted
  // kernel
  pl->off_part = o;
  o = align_up(o + (compact ? sizeof(long long) * 3 * (real_bytes / 4) * nn
                            : (size_t)real_bytes * kSlots * 3 * nn));
  pl->off_facc = o;      o = align_up(o + sizeof(float) * 3 * nn);
  pl->off_epart = o;     o = align_up(o + sizeof(double) * pl->n_tasks);
  pl->off_lj = o;        o = align_up(o + (size_t)real_bytes * 2 * kMaxTypes * kMaxTypes);
  pl->off_paircount = o; o = align_up(o + sizeof(int32_t) * 2 * nn);
  // binning with per-block LDS histograms when the grid fits in LDS
  pl->bin_blocks = 0;
  pl->bin_chunk = 0;
  if (n > 0 && cells <= kBinLdsCells) {
    int64_t chunk = (n + kBinMaxBlocks - 1) / kBinMaxBlocks;
    chunk = (chunk + kBinChunkUnit - 1) / kBinChunkUnit * kBinChunkUnit;
    pl->bin_chunk = chunk;
    pl->bin_blocks = (int)((n + chunk - 1) / chunk);
  }
  pl->off_bhist = o;     o = align_up(o + sizeof(int32_t) * (size_t)pl->bin_blocks * (cells + 1));
  pl->off_bstat = o;     o = align_up(o + sizeof(uint32_t) * (size_t)(pl->bin_blocks + 1));
  pl->off_order = o;     o = align_up(o + sizeof(int32_t) * cells);
  pl->off_cost = o;      o = align_up(o + sizeof(uint32_t) * cells);
  pl->off_zsplit = o;    o = align_up(o + sizeof(int32_t) * cells);
  pl->off_ukey = o;      o = align_up(o + sizeof(UKey) * nn);
  pl->off_upos = o;      o = align_up(o + (size_t)4 * real_bytes * nn);
  pl->off_kpart = o;     o = align_up(o + sizeof(double) * (size_t)ke_blocks(n));
  pl->total = o;
  return MD_OK;
}

template <typename Real>
SysArgs<Real> make_args(const md_params* p, const Plan& pl, int64_t n, const Real* pos,
                        const int32_t* type, const Real* q, Real* force, double* energy,
                        void* ws) {
  SysArgs<Real> a;
  char* b = (char*)ws;
  a.pos_in = pos;
  a.type_in = type;
  a.q_in = q;
  a.force_out = force;
  a.energy_out = energy;
  a.hdr = (WsHeader*)b;
  a.count = (int32_t*)(b + pl.off_count);
  a.start = (int32_t*)(b + pl.off_start);
  a.cell = (int32_t*)(b + pl.off_cell);
  a.rank = (int32_t*)(b + pl.off_rank);
  a.pos = (P4<Real>*)(b + pl.off_pos);
  a.hpre = (P4<Real>*)(b + pl.off_hpre);
  a.type = (int32_t*)(b + pl.off_type);
  a.perm = (int32_t*)(b + pl.off_perm);
  a.part = (Real*)(b + pl.off_part);
  a.facc = (float*)(b + pl.off_facc);
  a.epart = (double*)(b + pl.off_epart);
  a.lj = (Real*)(b + pl.off_lj);
  a.paircount = (int32_t*)(b + pl.off_paircount);
  a.acc64 = (long long*)(b + pl.off_part);   // the compacted kernel reuses the partial buffer
  a.bhist = (int32_t*)(b + pl.off_bhist);
  a.bstat = (uint32_t*)(b + pl.off_bstat);
  a.order = (int32_t*)(b + pl.off_order);
  a.cost = (uint32_t*)(b + pl.off_cost);
  a.zsplit = (int32_t*)(b + pl.off_zsplit);
  a.ukey = (UKey*)(b + pl.off_ukey);
  a.upos = (P4<Real>*)(b + pl.off_upos);
  a.bin_blocks = pl.bin_blocks;
  a.bin_chunk = pl.bin_chunk;
  a.n = n;
  a.n_cells = pl.n_cells;
  a.n_tasks = pl.n_tasks;
  a.nx = pl.dims[0];
  a.ny = pl.dims[1];
  a.nz = pl.dims[2];
  a.n_types = p->n_types;
  for (int d = 0; d < 3; ++d) {
    a.L[d] = (Real)p->box[d];
    a.inv_w[d] = (Real)((double)pl.dims[d] / (double)a.L[d]);
  }
  const double rc2 = p->r_cut * p->r_cut, rs2 = p->r_switch * p->r_switch;
  a.rc2 = (Real)rc2;
  a.rs2 = (Real)rs2;
  a.inv_sw = p->r_switch < p->r_cut ? (Real)(1.0 / (rc2 - rs2)) : Real(0);
  a.coulomb_k = (Real)p->coulomb_k;
  a.ewald_alpha = (p->flags & MD_COULOMB_EWALD) ? (Real)p->ewald_alpha : Real(0);
  a.flags = p->flags;
  a.compact = uses_compact(p, (int)sizeof(Real)) ? 1 : 0;
  a.half_shell =
      (a.compact && !(p->flags & (MD_ACCUM_F32_ATOMIC | MD_PAIR_FULL_SHELL))) ? 1 : 0;
  a.fs_split = a.compact ? md_fs_split(p->flags, pl.n_cells) : 1;
  return a;
}

template SysArgs<float> make_args<float>(const md_params*, const Plan&, int64_t, const float*,
                                         const int32_t*, const float*, float*, double*, void*);
template SysArgs<double> make_args<double>(const md_params*, const Plan&, int64_t,
                                           const double*, const int32_t*, const double*,
                                           double*, double*, void*);

// Synchronous argument checks of one force call; fills the plan.
template <typename Real>
static md_status check_call(const md_params* p, int64_t n, const Real* pos, const int32_t* type,
                            const Real* q, const Real* force, const double* energy,
                            const void* ws, size_t ws_bytes, Plan* pl) {
  md_status s = make_plan(p, n, (int)sizeof(Real), pl);
  if (s != MD_OK) return s;
  if (sizeof(Real) == 8 && (p->flags & MD_PAIR_DRAIN_MASK)) return MD_ERR_INVALID_ARG;
  // float64 with float32 atomics takes the predicated kernel, which has no Ewald form
  if (sizeof(Real) == 8 && (p->flags & MD_COULOMB_EWALD) && (p->flags & MD_ACCUM_F32_ATOMIC))
    return MD_ERR_INVALID_ARG;
  if (!energy || ((uintptr_t)energy & 7)) return MD_ERR_INVALID_ARG;
  if (n > 0) {
    if (!pos || !type || !q || !force) return MD_ERR_INVALID_ARG;
    if (((uintptr_t)pos | (uintptr_t)q | (uintptr_t)force) & (sizeof(Real) - 1))
      return MD_ERR_INVALID_ARG;
    if ((uintptr_t)type & 3) return MD_ERR_INVALID_ARG;
  }
  if (!ws || ((uintptr_t)ws & 255) || ws_bytes < pl->total) return MD_ERR_WORKSPACE;
  return MD_OK;
}

// Systems that may share one batched launch: same flags and the same type table.
static bool same_kind(const md_params* x, const md_params* y) {
  if (x->flags != y->flags || x->n_types != y->n_types || x->r_cut != y->r_cut ||
      x->r_switch != y->r_switch || x->coulomb_k != y->coulomb_k ||
      ((x->flags & MD_COULOMB_EWALD) && x->ewald_alpha != y->ewald_alpha))
    return false;
  for (int t = 0; t < x->n_types; ++t)
    if (x->sigma[t] != y->sigma[t] || x->epsilon[t] != y->epsilon[t]) return false;
  return true;
}

static md_status launch_batch(const Batch<float>& b, const md_params* p, hipStream_t st) {
  if (b.n == 0) return MD_OK;
  if (launch_binning_batch(b, make_type_table(p), st) != hipSuccess) return MD_ERR_HIP;
  if (launch_pair_fs_batch(b, st) != hipSuccess) return MD_ERR_HIP;
  if (launch_finalize_batch(b, st) != hipSuccess) return MD_ERR_HIP;
  return MD_OK;
}

template <typename Real>
static md_status forces_impl(const md_params* p, int64_t n, const Real* pos,
                             const int32_t* type, const Real* q, Real* force, double* energy,
                             void* ws, size_t ws_bytes, void* stream,
                             uint32_t stages = MD_STAGE_ALL) {
  if (stages & ~(uint32_t)MD_STAGE_ALL) return MD_ERR_INVALID_ARG;
  Plan pl;
  md_status s = check_call<Real>(p, n, pos, type, q, force, energy, ws, ws_bytes, &pl);
  if (s != MD_OK) return s;
  SysArgs<Real> a = make_args<Real>(p, pl, n, pos, type, q, force, energy, ws);
  hipStream_t st = (hipStream_t)stream;
  if ((stages & MD_STAGE_BIN) && launch_binning<Real>(a, make_type_table(p), st) != hipSuccess)
    return MD_ERR_HIP;
  if ((stages & MD_STAGE_PAIR) && launch_pair<Real>(a, st) != hipSuccess) return MD_ERR_HIP;
  if ((stages & MD_STAGE_FINALIZE) && launch_finalize<Real>(a, st) != hipSuccess)
    return MD_ERR_HIP;
  return MD_OK;
}

}  // namespace md

extern "C" {

size_t md_workspace_bytes(const md_params* p, int64_t n_atoms, int double_precision) {
  md::Plan pl;
  if (md::make_plan(p, n_atoms, double_precision ? 8 : 4, &pl) != MD_OK) return 0;
  return pl.total;
}

md_status md_workspace_layout(const md_params* p, int64_t n_atoms, int double_precision,
                              md_layout* out) {
  if (!out) return MD_ERR_INVALID_ARG;
  md::Plan pl;
  md_status s = md::make_plan(p, n_atoms, double_precision ? 8 : 4, &pl);
  if (s != MD_OK) return s;
  for (int d = 0; d < 3; ++d) out->dims[d] = pl.dims[d];
  out->n_cells = pl.n_cells;
  out->cell_start = pl.off_start;
  out->perm = pl.off_perm;
  out->pair_count = pl.off_paircount;
  out->energy_partials = pl.off_epart;
  out->n_energy_partials =
      md::uses_compact(p, double_precision ? 8 : 4)
          ? pl.n_cells * md::md_fs_split(p->flags, pl.n_cells)
          : pl.n_tasks;
  out->z_split = pl.off_zsplit;
  out->total_bytes = pl.total;
  return MD_OK;
}

md_status md_forces_f32(const md_params* p, int64_t n_atoms, const float* d_pos,
                        const int32_t* d_type, const float* d_charge, float* d_force,
                        double* d_energy, void* d_ws, size_t ws_bytes, void* stream) {
  return md::forces_impl<float>(p, n_atoms, d_pos, d_type, d_charge, d_force, d_energy, d_ws,
                                ws_bytes, stream);
}

md_status md_forces_f32_stages(const md_params* p, int64_t n_atoms, const float* d_pos,
                               const int32_t* d_type, const float* d_charge, float* d_force,
                               double* d_energy, void* d_ws, size_t ws_bytes, uint32_t stages,
                               void* stream) {
  return md::forces_impl<float>(p, n_atoms, d_pos, d_type, d_charge, d_force, d_energy, d_ws,
                                ws_bytes, stream, stages);
}

md_status md_forces_f64(const md_params* p, int64_t n_atoms, const double* d_pos,
                        const int32_t* d_type, const double* d_charge, double* d_force,
                        double* d_energy, void* d_ws, size_t ws_bytes, void* stream) {
  return md::forces_impl<double>(p, n_atoms, d_pos, d_type, d_charge, d_force, d_energy, d_ws,
                                 ws_bytes, stream);
}

md_status md_forces_f32_noalloc(const md_params* p, int64_t n_atoms, const float* d_pos,
                                const int32_t* d_type, const float* d_charge, float* d_force,
                                double* d_energy, uint32_t* d_status, void* stream) {
  md::Plan pl;
  // every argument check, the size limit included, before any HIP call
  md_status s = md::make_plan(p, n_atoms, 4, &pl);
  if (s != MD_OK) return s;
  if (pl.total > md::kScratchBytes) return MD_ERR_CAPACITY;
  if (d_status && ((uintptr_t)d_status & 3)) return MD_ERR_INVALID_ARG;
  // pointer checks of md_forces_f32 (the workspace is checked against a stand-in with the
  // scratch array's size and alignment)
  s = md::check_call<float>(p, n_atoms, d_pos, d_type, d_charge, d_force, d_energy,
                            (const void*)(uintptr_t)256, md::kScratchBytes, &pl);
  if (s != MD_OK) return s;
  void* ws = nullptr;
  s = md::noalloc_scratch(&ws);
  if (s != MD_OK) return s;
  s = md::forces_impl<float>(p, n_atoms, d_pos, d_type, d_charge, d_force, d_energy, ws,
                             md::kScratchBytes, stream);
  if (s != MD_OK || !d_status) return s;
  hipLaunchKernelGGL(md::k_copy_status, dim3(1), dim3(1), 0, (hipStream_t)stream,
                     (const md::WsHeader*)ws, d_status);
  return hipGetLastError() == hipSuccess ? MD_OK : MD_ERR_HIP;
}

md_status md_run_vv_f32(const md_params* p, int64_t n_atoms, float* d_pos, float* d_vel,
                        const int32_t* d_type, const float* d_charge, const float* d_inv_mass,
                        float* d_force, double dt_fs, int32_t n_steps, double* d_energies,
                        void* d_ws, size_t ws_bytes, void* stream) {
  if (n_steps < 0 || !isfinite(dt_fs)) return MD_ERR_INVALID_ARG;
  md::Plan pl;
  md_status s = md::check_call<float>(p, n_atoms, d_pos, d_type, d_charge, d_force, d_energies,
                                      d_ws, ws_bytes, &pl);
  if (s != MD_OK) return s;
  if (n_atoms > 0 && (!d_vel || !d_inv_mass || (((uintptr_t)d_vel | (uintptr_t)d_inv_mass) & 3)))
    return MD_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  // the box rounded once to float32, as the force path has it
  const float L[3] = {(float)p->box[0], (float)p->box[1], (float)p->box[2]};
  const float dt = (float)dt_fs, h = (float)(0.5 * dt_fs);
  double* kpart = (double*)((char*)d_ws + pl.off_kpart);
  for (int32_t k = 0; k < n_steps; ++k) {
    if (md::launch_vv_kick_drift(n_atoms, d_pos, d_vel, d_force, d_inv_mass, h, dt, L, st) !=
        hipSuccess)
      return MD_ERR_HIP;
    s = md::forces_impl<float>(p, n_atoms, d_pos, d_type, d_charge, d_force, d_energies + 2 * k,
                               d_ws, ws_bytes, stream);
    if (s != MD_OK) return s;
    if (md::launch_vv_kick(n_atoms, d_vel, d_force, d_inv_mass, h, kpart, d_energies + 2 * k + 1,
                           st) != hipSuccess)
      return MD_ERR_HIP;
  }
  return MD_OK;
}

md_status md_forces_batched(const md_system* sys, int32_t n_sys, void* stream) {
  if (n_sys < 0 || (n_sys > 0 && !sys)) return MD_ERR_INVALID_ARG;
  for (int32_t k = 0; k < n_sys; ++k) {
    md::Plan pl;
    md_status s = md::check_call<float>(&sys[k].p, sys[k].n_atoms, sys[k].d_pos, sys[k].d_type,
                                        sys[k].d_charge, sys[k].d_force, sys[k].d_energy,
                                        sys[k].d_ws, sys[k].ws_bytes, &pl);
    if (s != MD_OK) return s;
  }
  // Systems binned through LDS histograms and forced by the compacted kernel go in
  // batches of up to kBatchMax systems of one kind, in input order; any other system is
  // evaluated on its own.
  hipStream_t st = (hipStream_t)stream;
  md::Batch<float> b;
  b.n = 0;
  const md_params* kind = nullptr;
  for (int32_t k = 0; k < n_sys; ++k) {
    md::Plan pl;
    md::make_plan(&sys[k].p, sys[k].n_atoms, 4, &pl);
    const bool batchable = sys[k].n_atoms > 0 && pl.bin_blocks > 0 &&
                           !(sys[k].p.flags & MD_PAIR_PREDICATED);
    if (!batchable) {
      md_status s = md_forces_f32(&sys[k].p, sys[k].n_atoms, sys[k].d_pos, sys[k].d_type,
                                  sys[k].d_charge, sys[k].d_force, sys[k].d_energy, sys[k].d_ws,
                                  sys[k].ws_bytes, stream);
      if (s != MD_OK) return s;
      continue;
    }
    if (b.n == md::kBatchMax || (b.n > 0 && !md::same_kind(kind, &sys[k].p))) {
      md_status s = md::launch_batch(b, kind, st);
      if (s != MD_OK) return s;
      b.n = 0;
    }
    if (b.n == 0) kind = &sys[k].p;
    b.sys[b.n++] = md::make_args<float>(&sys[k].p, pl, sys[k].n_atoms, sys[k].d_pos,
                                        sys[k].d_type, sys[k].d_charge, sys[k].d_force,
                                        sys[k].d_energy, sys[k].d_ws);
  }
  return md::launch_batch(b, kind, st);
}

md_status md_read_device_status(const void* d_ws, void* stream, uint32_t* bits) {
  if (!d_ws || !bits) return MD_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  uint32_t v = 0;
  if (hipMemcpyAsync(&v, d_ws, sizeof(v), hipMemcpyDeviceToHost, st) != hipSuccess)
    return MD_ERR_HIP;
  if (hipStreamSynchronize(st) != hipSuccess) return MD_ERR_HIP;
  *bits = v;
  return MD_OK;
}

md_status md_read_diag(const void* d_ws, void* stream, uint64_t counters[5]) {
  if (!d_ws || !counters) return MD_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  md::WsHeader h;
  if (hipMemcpyAsync(&h, d_ws, sizeof(h), hipMemcpyDeviceToHost, st) != hipSuccess)
    return MD_ERR_HIP;
  if (hipStreamSynchronize(st) != hipSuccess) return MD_ERR_HIP;
  for (int k = 0; k < 5; ++k) counters[k] = h.diag[k];
  return MD_OK;
}

md_status md_read_clock(const void* d_ws, void* stream, double* ghz) {
  if (!d_ws || !ghz) return MD_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  md::WsHeader h;
  if (hipMemcpyAsync(&h, d_ws, sizeof(h), hipMemcpyDeviceToHost, st) != hipSuccess)
    return MD_ERR_HIP;
  if (hipStreamSynchronize(st) != hipSuccess) return MD_ERR_HIP;
  *ghz = h.clock[1] ? 0.1 * (double)h.clock[0] / (double)h.clock[1] : 0.0;
  return MD_OK;
}

const char* md_status_string(md_status s) {
  switch (s) {
    case MD_OK: return "ok";
    case MD_ERR_INVALID_ARG: return "invalid argument";
    case MD_ERR_BOX_TOO_SMALL: return "box too small: fewer than 2 cells of edge >= r_cut";
    case MD_ERR_WORKSPACE: return "workspace missing, misaligned or too small";
    case MD_ERR_HIP: return "HIP runtime error";
    case MD_ERR_DEVICE_STATUS: return "device status word set";
    case MD_ERR_CAPACITY: return "problem exceeds an internal limit";
  }
  return "unknown status";
}

}  // extern "C"
