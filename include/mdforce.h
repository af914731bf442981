/*
 * mdforce.h -- C ABI of the MI355X (gfx950) short-range non-bonded force library.
 *
 * The library evaluates one iteration of the short-range non-bonded force of
 * molecular dynamics, the critical path named in Section 2.1 of Cong, Fang,
 * Kianinejad, Wei, "Revisiting FPGA Acceleration of Molecular Dynamics Simulation
 * with Dynamic Data Flow Behavior in High-Level Synthesis" (arXiv:1611.04474):
 *
 *   - Lennard-Jones force, Eq. 1:  F = (A/|r|^14 - B/|r|^8) r,
 *     with A = 48 eps_ij s_ij^12 and B = 24 eps_ij s_ij^6 from per-type sigma and
 *     epsilon by Lorentz-Berthelot mixing (s_ij = (s_i+s_j)/2, eps_ij = sqrt(eps_i eps_j));
 *   - Coulomb force, Eq. 2:  F = k q_i q_j / |r|^3 r;
 *   - the cutoff of Section 2.1: a pair interacts only if |r|^2 < r_cut^2;
 *   - the cell list of Section 2.1 (Fig. 2, Algorithm 1): space is cut into cells of
 *     edge at least r_cut and each atom meets only the atoms of its 3x3x3 cells.
 *
 * r is x_i - x_j (the force on atom i is +f r; a positive f pushes i and j apart).
 * The whole pair energy e = c12/r^12 - c6/r^6 + k q_i q_j / r (c12 = 4 eps s^12,
 * c6 = 4 eps s^6) is multiplied by the switch S(u), u = r^2, which is 1 up to
 * r_switch^2 and (rc2-u)^2 (rc2+2u-3rs2)/(rc2-rs2)^3 between r_switch^2 and r_cut^2;
 * forces are minus the gradient of S e. r_switch == r_cut turns switching off.
 * Units: Angstrom, elementary charge, kcal/mol.
 *
 * Conventions for every call:
 *   - d_ pointers are device pointers on the current HIP device; h_ pointers, and
 *     the sigma/epsilon arrays inside md_params, are host pointers.
 *   - The caller owns every buffer, including the workspace; the library allocates
 *     no device memory and keeps no global state, so calls with distinct
 *     workspaces may run concurrently. The one exception is md_forces_f32_noalloc,
 *     which uses a workspace of the library's own, one per device.
 *   - Argument checks are synchronous and return an md_status; nothing is enqueued
 *     when a check fails. Work is enqueued on `stream` (a hipStream_t, or NULL for
 *     the default stream) and outputs are valid once the stream reaches the call.
 *   - Conditions found on the device (NaN or out-of-range positions, bad type
 *     indices, fixed-point overflow) set bits of a sticky status word in the
 *     workspace, read with md_read_device_status.
 */
#ifndef MDFORCE_H
#define MDFORCE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MD_OK = 0,
  MD_ERR_INVALID_ARG = -1,   /* null pointer, n_atoms < 0, bad flags, r_switch > r_cut ... */
  MD_ERR_BOX_TOO_SMALL = -2, /* some box edge gives fewer than 2 cells of edge >= r_cut */
  MD_ERR_WORKSPACE = -3,     /* workspace null, misaligned (256 B) or smaller than needed */
  MD_ERR_HIP = -4,           /* a HIP runtime call failed */
  MD_ERR_DEVICE_STATUS = -5, /* reserved for callers that fold the status word in */
  MD_ERR_CAPACITY = -6       /* problem exceeds an internal limit (cells, atoms, types) */
} md_status;

/* md_params.flags */
enum {
  MD_ACCUM_FIXED64 = 0,         /* default: per-atom sums in 64-bit fixed point (2^-28 kcal/mol/A
                                   in float32; hi 2^-20 + lo 2^-72 in float64) */
  MD_ACCUM_F32_ATOMIC = 1 << 0, /* per-atom sums in float32: with float32 atomics (order-
                                   dependent) in the predicated kernels; on the compacted path
                                   by the full-shell kernel, which owns each atom in one wave,
                                   as a fixed-order float32 sum */
  MD_COULOMB_TRUNCATED = 1 << 1,/* switch only the LJ energy; Coulomb is Eq. 2 up to r_cut */
  MD_DIAG_COUNTERS = 1 << 2,    /* count candidates, filter passes and per-atom partners */
  MD_PAIR_PREDICATED = 1 << 3,  /* evaluate the force under the cutoff predicate, without
                                   compacting passing pairs (the uncompacted data flow) */
  MD_COULOMB_EWALD = 1 << 7,    /* Coulomb inside the cutoff is the real-space term of an Ewald
                                   sum, k q_i q_j erfc(alpha r)/r with alpha = ewald_alpha; only
                                   the LJ energy is switched. The rest of the Coulomb energy (its
                                   beyond-cutoff part, which Section 2.1 leaves to an O(N)
                                   approximation outside the short-range kernel) comes from
                                   md_ewald_recip_f32. Compacted kernel only (not with
                                   MD_PAIR_PREDICATED, MD_COULOMB_TRUNCATED, or float64 with
                                   MD_ACCUM_F32_ATOMIC) */
  MD_PAIR_FULL_SHELL = 1 << 4   /* compacted float32 path: evaluate every pair from both of
                                   its atoms, in the loop order of Algorithm 1 (Section 2.1),
                                   each atom's sum kept by one wave, no atomics. Default: each
                                   pair once (Newton's third law), the partner's share added
                                   with 64-bit integer atomics, which give the same sum in
                                   any order */
};

/* md_params.flags bits 5-6: force batches of 64 pairs drained together from a full FIFO
 * by the compacted half-shell kernel with the whole energy switched -- the candidate
 * batches per force pass, swept like the distance PEs per force PE of Section 5.2
 * (Table 6). 0 keeps the default depth 2; MD_PAIR_DRAIN(d) selects d = 1, 3 or 4. Any other
 * configuration (float64, predicated, full shell, float32 sums, Coulomb truncated,
 * r_switch == r_cut) accepts only 0 and returns MD_ERR_INVALID_ARG otherwise. */
#define MD_PAIR_DRAIN_MASK (3u << 5)
#define MD_PAIR_DRAIN(d) ((uint32_t)((d) == 1 ? 1 : (d) == 3 ? 2 : (d) == 4 ? 3 : 0) << 5)

/* md_params.flags bits 8-9: workgroups of the compacted kernel per home cell, each taking
 * every s-th group of the cell's home atoms (the work units of the loop over home atoms of
 * Algorithm 1, spread over more compute units). 0 chooses automatically (4 on grids of at
 * most 64 cells, 2 up to 128, else 1); MD_PAIR_SPLIT(s) forces s = 1, 2 or 4. Results are the
 * same bits for every s. Not with MD_PAIR_PREDICATED (MD_ERR_INVALID_ARG). */
#define MD_PAIR_SPLIT_MASK (3u << 8)
#define MD_PAIR_SPLIT(s) ((uint32_t)((s) == 1 ? 1 : (s) == 2 ? 2 : (s) == 4 ? 3 : 0) << 8)

/* Device status bits (sticky until the next force call on the workspace). */
enum {
  MD_STATUS_NAN = 1u << 0,          /* a position is NaN */
  MD_STATUS_OUT_OF_BOX = 1u << 1,   /* a coordinate lies outside [-L, 2L) */
  MD_STATUS_BAD_TYPE = 1u << 2,     /* a type index outside [0, n_types) */
  MD_STATUS_FIXED_OVERFLOW = 1u << 3/* a force does not fit the 64-bit fixed-point range */
};

/* Problem description. The box is orthorhombic and periodic on all three axes;
 * each edge must give at least two cells of edge >= r_cut (so L >= 2 r_cut, with a
 * 1e-3 A margin: n_d = floor(L_d/r_cut), reduced by one when L_d/n_d - r_cut < 1e-3).
 * The float32 entry points use every box edge rounded once to float32. */
typedef struct {
  double box[3];          /* A */
  double r_cut;           /* A, > 0 */
  double r_switch;        /* A, 0 < r_switch <= r_cut */
  double coulomb_k;       /* kcal*A/(mol*e^2), e.g. 332.0636 */
  int32_t n_types;        /* 1 .. 64 */
  const double* sigma;    /* host [n_types], A */
  const double* epsilon;  /* host [n_types], kcal/mol, >= 0 */
  uint32_t flags;         /* MD_* flags above */
  double ewald_alpha;     /* 1/A, > 0: Ewald splitting parameter (MD_COULOMB_EWALD) */
} md_params;

/* Library support (no passage of the paper defines it: the caller owns all device memory).
 * Bytes of device workspace needed by md_forces_f32 (double_precision = 0) or
 * md_forces_f64 (double_precision = 1) for n_atoms atoms with p->flags (the flags
 * choose the pair kernel, whose per-atom buffers differ in size). Returns 0 when the
 * parameters are invalid. The workspace must be 256-byte aligned; its contents
 * need no initialisation. Between calls they are scratch, except that the
 * compacted kernel leaves each home cell's measured time there: the next call on the
 * same workspace and cell grid (of at most 1024 cells) launches the cells longest first
 * by those times. They only steer scheduling, never a result, so any contents are
 * valid. */
size_t md_workspace_bytes(const md_params* p, int64_t n_atoms, int double_precision);

/*
 * One evaluation of the short-range non-bonded forces (Section 2.1, Algorithm 1).
 *   d_pos     [n_atoms][3] float32, x,y,z interleaved; coordinates in [-L, 2L) are
 *             wrapped into the box with one float32 add or subtract of L.
 *   d_type    [n_atoms] int32 type indices in [0, n_types).
 *   d_charge  [n_atoms] float32 charges (e).
 *   d_force   [n_atoms][3] float32 output, in the caller's atom order, kcal/mol/A.
 *   d_energy  [1] float64 output, total pair energy over unique pairs, kcal/mol.
 *   d_ws      workspace of at least md_workspace_bytes(p, n_atoms, 0) bytes.
 * n_atoms == 0 enqueues a zero energy only. Pair arithmetic is float32; per-atom
 * sums are 64-bit fixed point unless MD_ACCUM_F32_ATOMIC; the energy is an exact sum of
 * 64-bit fixed-point partials (2^-24 kcal/mol) after the compacted kernel, and a float64
 * sum in a fixed order after the predicated one.
 */
md_status md_forces_f32(const md_params* p, int64_t n_atoms, const float* d_pos,
                        const int32_t* d_type, const float* d_charge, float* d_force,
                        double* d_energy, void* d_ws, size_t ws_bytes, void* stream);

/* Library support (no passage of the paper: the stages are those of Section 2.1's
 * iteration, binning, pair forces, per-atom sums, enqueued separately).
 * Stages of one evaluation, for callers that time or interleave them:
 *   MD_STAGE_BIN       clear counters, wrap positions, counting-sort binning;
 *   MD_STAGE_PAIR      cutoff filter and force over all cell-pair tasks;
 *   MD_STAGE_FINALIZE  per-atom sums in the caller's order and the total energy.
 * Enqueuing the stages in this order on one workspace and stream gives exactly the
 * result of md_forces_f32 with the same arguments; the arguments must not change
 * between the stages of one evaluation. */
enum { MD_STAGE_BIN = 1, MD_STAGE_PAIR = 2, MD_STAGE_FINALIZE = 4, MD_STAGE_ALL = 7 };

md_status md_forces_f32_stages(const md_params* p, int64_t n_atoms, const float* d_pos,
                               const int32_t* d_type, const float* d_charge, float* d_force,
                               double* d_energy, void* d_ws, size_t ws_bytes,
                               uint32_t stages, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): md_forces_f32 with the library's own
 * workspace instead of a caller-owned one, so the call allocates nothing.
 *   - The workspace is a static device array of MD_NOALLOC_MAX_WORKSPACE_BYTES (32 MiB)
 *     per device, created when the library's code is first used on that device and held
 *     until the process ends. Its device address is looked up once per device, on the
 *     first call with that device current.
 *   - Systems whose md_workspace_bytes(p, n_atoms, 0) exceeds that size are rejected with
 *     MD_ERR_CAPACITY before anything is enqueued (at 8 atom types about 230,000 atoms
 *     of the 0.1 atoms/A^3 systems). Other argument errors as for md_forces_f32.
 *   - Every call on one device uses that device's one array: calls that overlap on one
 *     device (other streams, other host threads) race and give undefined results;
 *     serialise them. Each call starts from whatever the previous one left, which is
 *     valid: nothing in the workspace needs initialisation.
 *   - d_status, if not NULL, is caller-owned device memory (4 bytes, 4-byte aligned) that
 *     receives the call's device status word (MD_STATUS_* bits) in stream order.
 * Other arguments, outputs and the asynchrony as for md_forces_f32. */
#define MD_NOALLOC_MAX_WORKSPACE_BYTES (32u << 20)
md_status md_forces_f32_noalloc(const md_params* p, int64_t n_atoms, const float* d_pos,
                                const int32_t* d_type, const float* d_charge, float* d_force,
                                double* d_energy, uint32_t* d_status, void* stream);

/* Same as md_forces_f32 with float64 positions, charges, forces and pair arithmetic
 * throughout (the FP64-everywhere form of Section 2.1's computation): the same compacted
 * kernel, instantiated for float64, with the cutoff test on a plain float64 evaluation of
 * dx^2 + dy^2 + dz^2. Per-atom sums and the energy are exact integer sums of a two-word
 * fixed point (hi 2^-20 + lo 2^-72 kcal/mol/A), so results are the same bits on every run;
 * MD_PAIR_FULL_SHELL selects the full shell as in float32. With MD_PAIR_PREDICATED (or
 * MD_ACCUM_F32_ATOMIC) the predicated kernel runs instead, its per-atom partials added in
 * float64 in a fixed slot order (float32 atomics with MD_ACCUM_F32_ATOMIC). */
md_status md_forces_f64(const md_params* p, int64_t n_atoms, const double* d_pos,
                        const int32_t* d_type, const double* d_charge, double* d_force,
                        double* d_energy, void* d_ws, size_t ws_bytes, void* stream);

/* Ewald reciprocal-space sum: the Coulomb energy and forces beyond the short-range
 * kernel. Section 2.1 splits the non-bonded work at the cutoff and leaves the Coulomb part
 * beyond it to an approximation outside the short-range kernel; with MD_COULOMB_EWALD the
 * short-range call evaluates the screened term k q_i q_j erfc(alpha r)/r inside the cutoff
 * and this call the rest of the periodic Coulomb sum:
 *   E = k/(2V) sum_{kv != 0} (4 pi/|kv|^2) exp(-|kv|^2/(4 alpha^2)) |S(kv)|^2
 *       - k alpha/sqrt(pi) sum_j q_j^2 - k pi Q^2/(2 V alpha^2),
 *   S(kv) = sum_j q_j exp(i kv . r_j),  kv = 2 pi (mx/Lx, my/Ly, mz/Lz), |m_d| <= kmax[d],
 * (reciprocal sum, self term, neutralising background for net charge Q) and the forces
 * -dE/dr_i. alpha is p->ewald_alpha (> 0); the box is p->box rounded to float32, r_cut and
 * the type table are not used. Each atom's phase is exact modulo one turn (32-bit
 * fixed-point fractional coordinates); sums run in float32 within tiles and float64
 * across them, in a fixed order.
 *   d_pos     [n_atoms][3] float32, any coordinates (the sum is periodic)
 *   d_charge  [n_atoms] float32
 *   kmax      host int32[3], each 0..255, not all 0
 *   d_force   [n_atoms][3] float32 out, caller order: written, or added to when
 *             accumulate != 0 (e.g. onto the short-range forces)
 *   d_energy  [1] float64 out: reciprocal + self + background energy
 *   d_ws      workspace of md_ewald_workspace_bytes(p, n_atoms, kmax) bytes, 256-B aligned;
 *             its first word is a status word (MD_STATUS_NAN for a NaN position or charge),
 *             read with md_read_device_status
 * Errors: MD_ERR_INVALID_ARG (alpha, box, kmax, pointers), MD_ERR_WORKSPACE, MD_ERR_HIP.
 * md_ewald_workspace_bytes returns 0 for invalid arguments. */
size_t md_ewald_workspace_bytes(const md_params* p, int64_t n_atoms, const int32_t kmax[3]);
md_status md_ewald_recip_f32(const md_params* p, int64_t n_atoms, const float* d_pos,
                             const float* d_charge, const int32_t kmax[3], float* d_force,
                             double* d_energy, int32_t accumulate, void* d_ws, size_t ws_bytes,
                             void* stream);

/* One system of a batch (float32 path). Every field as in md_forces_f32. */
typedef struct {
  md_params p;
  int64_t n_atoms;
  const float* d_pos;
  const int32_t* d_type;
  const float* d_charge;
  float* d_force;
  double* d_energy;
  void* d_ws;
  size_t ws_bytes;
} md_system;

/* Serving support (no passage of the paper: it evaluates one system at a time).
 * Evaluates n_sys independent systems, each in its own periodic box with its own
 * workspace, as one launch sequence on `stream`: each kernel of the path is
 * launched once for the whole batch. Results are identical to one md_forces_f32
 * call per system. Argument errors of any system fail the whole call before
 * anything is enqueued. */
md_status md_forces_batched(const md_system* systems, int32_t n_sys, void* stream);

/* Motion update around the force call: n_steps velocity-Verlet steps of dt fs on
 * device-resident state (each MD iteration computes the forces on every atom, then updates
 * the atoms' motion: Section 1, Section 2.1; the paper names no integrator). Per step:
 *   v += (dt/2) F/m;  x += dt v, wrapped into [0, L) by one add or subtract of L;
 *   F = the force path of md_forces_f32 at the new x;  v += (dt/2) F/m.
 * Units: A, fs, amu, kcal/mol; F/m in (kcal/mol/A)/amu is 4.184e-4 A/fs^2.
 *   d_pos      float32 [n][3], in/out: positions (caller order), as for md_forces_f32
 *   d_vel      float32 [n][3], in/out: velocities, A/fs
 *   d_inv_mass float32 [n]: 1/m per atom, 1/amu (0 pins an atom)
 *   d_force    float32 [n][3], in: the forces at d_pos (from md_forces_f32 with the same
 *              parameters); out: the forces at the final positions
 *   d_energies double [n_steps][2], out: potential and kinetic energy (kcal/mol) after
 *              each step, the kinetic energy summed in a fixed order
 * Workspace, stream, status word and errors as for md_forces_f32; dt must be finite and
 * n_steps >= 0 (0 does nothing). All device pointers are caller-owned. */
md_status md_run_vv_f32(const md_params* p, int64_t n_atoms, float* d_pos, float* d_vel,
                        const int32_t* d_type, const float* d_charge, const float* d_inv_mass,
                        float* d_force, double dt_fs, int32_t n_steps, double* d_energies,
                        void* d_ws, size_t ws_bytes, void* stream);

/* Serving runtime support (no passage of the paper: moving requests in and out).
 * Copies n_segs byte ranges, each between device memory and pinned (hipHostMalloc) host
 * memory or within device memory, with kernel launches on `stream` (one per 128 segments):
 * the copies are enqueued in stream order like a kernel, without the runtime's copy
 * engines. Segments of 0 bytes are skipped; the ranges of one call must not overlap. All
 * memory is caller-owned and stays valid until the stream reaches the call.
 * Errors: MD_ERR_INVALID_ARG (n_segs < 0, a null array, or a null address in a non-empty
 * segment), MD_ERR_HIP if a launch fails. */
typedef struct {
  void* dst;
  const void* src;
  size_t bytes;
} md_copy_segment;

md_status md_copy_segments(const md_copy_segment* segs, int32_t n_segs, void* stream);

/* Library support (no passage of the paper: error reporting).
 * Copies the sticky device status word of a workspace to *bits (MD_STATUS_* bits).
 * Synchronises `stream`. */
md_status md_read_device_status(const void* d_ws, void* stream, uint32_t* bits);

/* Measurement support. No passage defines the call; the counters measure the quantities
 * of Section 5 (candidates against pairs that pass the cutoff, and the force stage's
 * utilisation that Table 7 reports for the force PE).
 * Diagnostic counters of the last call with MD_DIAG_COUNTERS on this workspace, all
 * per unique pair:
 *   [0] candidate pairs of the cell list (every pair of atoms in neighbouring cells,
 *       Algorithm 1), the work a filter that tests them all would do;
 *   [1] pairs passing the filter stage (the conservative prefilter of the compacted
 *       kernel, the cutoff test itself for the predicated one);
 *   [2] pairs inside the cutoff;
 *   [3] candidate pairs the filter stage actually examined (the compacted kernel skips
 *       neighbours outside an x-window of its home atoms; equal to [0] otherwise);
 *   [4] lanes that went through the force arithmetic (the compacted kernel's dense
 *       passes; every candidate for the predicated kernel), so [2] / [4] is the force
 *       stage's lane utilisation.
 * For the float32 compacted kernel, which sees every pair from both atoms, [1], [3] and
 * [4] are half of its per-atom counts. Synchronises `stream`. */
md_status md_read_diag(const void* d_ws, void* stream, uint64_t counters[5]);

/* Measurement support (no passage of the paper: the clock under load that scales the
 * roofline peak).
 * The shader clock, in GHz, at which the compacted pair kernel of the last call on this
 * workspace ran: each of its workgroups counts shader-clock cycles and ticks of the
 * constant 100 MHz counter over its run, and *ghz is the ratio of the two sums times
 * 0.1, i.e. the clock averaged over workgroup time. Scaling a peak rate quoted at the
 * nominal clock by *ghz / nominal gives the peak at the clock the kernel really ran at.
 * *ghz is 0 when no compacted pair kernel (float32 or float64) has run since the last
 * binning (the predicated kernel does not count). Errors: MD_ERR_INVALID_ARG for a null pointer,
 * MD_ERR_HIP if the copy fails. Synchronises `stream`. */
md_status md_read_clock(const void* d_ws, void* stream, double* ghz);

/* Library support (no passage of the paper, though the arrays are those of Section 2.2's
 * flat cell layout).
 * Layout of the workspace, for inspection of intermediate results. Offsets are in
 * bytes from the workspace start.
 *   cell_start: int32 [n_cells+1], first sorted index of each cell
 *   perm:       int32 [n_atoms], original index of each sorted atom
 *   pair_count: int32 [n_atoms], partners inside the cutoff (MD_DIAG_COUNTERS),
 *               in the caller's atom order
 *   energy_partials: per-workgroup energy sums, n_energy_partials of them: after the
 *               predicated kernel float64; after the compacted kernel exact integers,
 *               int64 in units of 2^-24 kcal/mol (float32) or two int64 words, hi 2^-20 +
 *               lo 2^-72 kcal/mol (float64), times 1/2 for the full shell
 *   z_split:    int32 [n_cells], atoms of each cell in its lower z half; a cell's sorted
 *               atoms are ordered by (z half, x, original index) */
typedef struct {
  int32_t dims[3];
  int64_t n_cells;
  size_t cell_start;
  size_t perm;
  size_t pair_count;
  size_t energy_partials;
  int64_t n_energy_partials;
  size_t z_split;
  size_t total_bytes;
} md_layout;

md_status md_workspace_layout(const md_params* p, int64_t n_atoms, int double_precision,
                              md_layout* out);

/* Library support (no passage of the paper: error reporting). Static description of a
 * status code. */
const char* md_status_string(md_status s);

#ifdef __cplusplus
}
#endif

#endif /* MDFORCE_H */
