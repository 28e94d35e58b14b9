/*
 * ephbte.h -- C ABI of the MI355X e-ph collision-integral library.
 *
 * The library evaluates the electron-phonon collision integral I[f](n,k) of
 * arXiv 2511.03683 (Results, "Collision integral, e-ph coupling matrix, and
 * scattering channels", Eq. 2) over a precomputed list of scattering
 * channels, and drives its two consumers: real-time BTE time stepping and the
 * iterative transport BTE (Results, "BTE for transport and ultrafast
 * dynamics", Eq. 1).  All arithmetic runs in HIP kernels on gfx950.
 *
 * Conventions shared by every call
 * --------------------------------
 * Units: energies eV, time fs, temperature K, velocity m/s, |g|^2 eV^2,
 *   I in 1/fs.  Constants: hbar = 0.6582119569 eV fs, k_B = 8.617333262e-5 eV/K.
 * States: S electronic states (n,k) inside the energy window.  State s has a
 *   linear k index state_k[s] = (k0*N1 + k1)*N2 + k2 on the k grid (N0,N1,N2).
 * Phonons: tables indexed [q][nu] (q-major, q linear on the q grid like k),
 *   n_modes <= 8.  The tables must be even in q (hw(-q) = hw(q), N(-q) = N(q)),
 *   as time-reversal symmetry gives; each orientation of a channel uses its own q.
 * Channel: an unordered state pair {i, j} plus a mode nu, with one |g|^2 value.
 *   It enters I(i) with partner j and q = k_j - k_i, and I(j) with partner i
 *   and q = k_i - k_j (Optimized GPU algorithm, step 1: each channel feeds two
 *   collision-integral elements).  k_j - k_i must be a q-grid vector
 *   (commensurate grids, Eq. 2 text).
 * Collision integral (Eq. 2 with Fermi's golden-rule occupation factors):
 *   I(d) = sum over channels touching d, partner p, mode nu, q = k_p - k_d:
 *     -(2 pi/hbar)(1/N_q) |g|^2 [ G(e_d - e_p + hw) F_abs + G(e_d - e_p - hw) F_em ]
 *   F_abs = f_d (1-f_p) N - f_p (1-f_d)(N+1),  F_em = f_d (1-f_p)(N+1) - f_p (1-f_d) N,
 *   G(x) = exp(-x^2 / (2 sigma^2)) / (sigma sqrt(2 pi)).
 * Precision: a plan is FP64 (EPHBTE_F64) or FP32 (EPHBTE_F32).  All device
 *   arrays passed to a plan (f, nph, I, gradients except gg2, x) have the
 *   plan's type; gg2 and transport outputs are FP64 always.
 * Batches: f and I hold B vectors of S values each, vector b at
 *   f + b*ldf (ldf >= S elements).  One phonon table serves all vectors.
 * Pointers: "host" pointers are read during the call only (the library keeps
 *   copies); "device" pointers are caller-owned HIP device memory on the
 *   plan's device, read or written by work enqueued on `stream`.
 * Streams: `stream` is a hipStream_t passed as void* (0 = null stream).  Work
 *   is enqueued asynchronously; calls that return host scalars synchronise.
 *   A plan's workspaces are shared by all its calls, so the library orders
 *   them: a call on a different stream than the plan's previous call first
 *   waits (device side) for that call's work.  Calls made while the caller is
 *   capturing the stream into a graph are not ordered this way.
 * Errors: every call returns a status and never throws.  Arguments are checked
 *   before any work is enqueued; on error nothing is enqueued and
 *   ephbte_last_error() (thread-local) describes the failure.
 * Determinism: results are bitwise reproducible run to run for a given plan
 *   and launch configuration.  Floating-point sums have a fixed order and use
 *   no atomics.  The single-copy passes (forward and reverse, layouts 2 and 3)
 *   add the partner side of each channel or pair (and, for the pair records
 *   in q order, the destination side too) with integer atomics on 64-bit
 *   fixed-point values; integer addition is associative, so those sums do
 *   not depend on the order of arrival.  The phonon-side rate uses no
 *   atomics.  The fixed-point scale is a power of two chosen per call from
 *   max |N| of the call's table, the largest sum of |g|^2 over one state's
 *   channels (and max |lambda| in the reverse pass); Fermi plans assume
 *   occupations f in [0, 1] (a caller's f outside that range, or RK stage
 *   inputs that leave it, can overflow the partner-side sums), Bose plans
 *   take max |n| of each pass's input into the scale.
 */
#ifndef EPHBTE_H
#define EPHBTE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ephbte_status;
#define EPHBTE_OK 0
#define EPHBTE_INVALID_ARGUMENT 1
#define EPHBTE_UNSUPPORTED_DTYPE 2
#define EPHBTE_OUT_OF_MEMORY 3
#define EPHBTE_HIP_ERROR 4
#define EPHBTE_NOT_CONVERGED 5
#define EPHBTE_NONFINITE 6
#define EPHBTE_PLAN_MISMATCH 7

#define EPHBTE_F32 1
#define EPHBTE_F64 2

typedef struct ephbte_plan_s *ephbte_plan;

/* Problem statement (paper: Eq. 2 and the scattering-channel paragraph that
 * follows it; energy window of Table 1).  All pointers are HOST pointers. */
typedef struct {
    int32_t n_states;          /* S >= 1, S < 2^29                                  */
    const int32_t *state_k;    /* [S] linear k index of each state                 */
    const int8_t *state_band;  /* [S] band of each state, or NULL (all band 0); only
                                  the field term uses it, to find a state's
                                  neighbours in its own band, and only where each
                                  (k, band) is held by one state                    */
    const double *eps;         /* [S] state energies (eV)                          */
    int32_t kgrid[3];          /* electron grid (N0,N1,N2)                         */
    int32_t qgrid[3];          /* phonon grid; kgrid[a] % qgrid[a] == 0, <= 1024   */
    int32_t n_modes;           /* 1..8                                             */
    const double *hw;          /* [Nq][n_modes] phonon energies (eV), >= 0         */
    int64_t n_channels;        /* >= 0, < 2^30                                     */
    const int32_t *ch_i;       /* [n_channels] state index, 0 <= i < S             */
    const int32_t *ch_j;       /* [n_channels] state index, j != i                 */
    const int8_t *ch_nu;       /* [n_channels] mode, 0 <= nu < n_modes             */
    const double *g2;          /* [n_channels] |g|^2 (eV^2), finite, >= 0          */
    double sigma;              /* Gaussian standard deviation (eV), > 0            */
    double n_q_norm;           /* N_q of Eq. 2 (full q-grid count), > 0            */
    int32_t dtype;             /* EPHBTE_F32 or EPHBTE_F64                         */
    int32_t device;            /* HIP device ordinal; -1 = current device          */
} ephbte_problem;

/* Tuning knobs of a plan (all optional: 0 keeps the plan's current value). */
typedef struct {
    int32_t chunk_entries;     /* max destination entries per workgroup chunk      */
    int32_t block_threads;     /* threads per workgroup: 64, 128, 256, 512         */
    int32_t xcd_map;           /* single-vector forward pass: 1 = each of the 8 XCDs
                                  takes a contiguous range of tiles (default),
                                  2 = tiles in plain order                         */
    int32_t batch_partners;    /* partner states per LDS sub-tile of the B >= 8 pass,
                                  16 .. 1024, within the device's LDS per workgroup */
    int32_t tile_entries;      /* target entries per workgroup tile of the B < 8
                                  passes (a tile never splits a chunk); -1 = the
                                  library's default                               */
    int32_t layout;            /* single-vector forward pass: 1 = every channel
                                  evaluated in both of its rows, 2 = once, from
                                  the row of its smaller state, one entry per
                                  channel, 3 = once, over pair records (all modes
                                  of a state pair together; the default when at
                                  least half of the records' mode slots hold a
                                  channel, else 2 is the default; both need the
                                  LDS per workgroup to allow them)                */
    int32_t fp64_exp;          /* FP64 Gaussians of the pair-record pass: 1 = table
                                  exponential (256 powers of 2^(1/256) in LDS,
                                  default), 2 = polynomial only (no LDS reads)   */
    int32_t table_order;       /* order of the {hw, N} table over the box of q
                                  differences: 1 = the modes of one q adjacent
                                  (one 16-byte row per mode, default),
                                  2 = one block per mode (a wave's gathers of
                                  one mode at neighbouring q share cache lines) */
    int32_t pair_window;       /* partner states per LDS window of the pair-record
                                  passes, 64 .. the most the LDS of a workgroup
                                  holds for the reverse pass (default 3072 FP64,
                                  4096 FP32)                                     */
    int32_t pair_threads;      /* threads per workgroup of the pair-record forward
                                  pass: 256, 512, 768 or 1024 (default)         */
    int32_t pair_order;        /* records of the pair-record passes' LDS tiles:
                                  1 = sorted by q = k_p - k_d (default: the lanes
                                  of a wave share rows of the {hw, N} table, and
                                  both sides of a pair are fixed-point sums),
                                  2 = by destination (the destination's side
                                  summed in registers)                         */
    int32_t pair_rows;         /* q order of pair_order 1: table rows per sort
                                  group, a power of 2 up to 65536 (default 1:
                                  sorted by q itself).  Larger groups keep more
                                  of a destination's records together, which
                                  makes the reverse pass's dL/d|g|^2 writes more
                                  contiguous when the caller lists channels by
                                  state pair, at some cost to the forward pass */
} ephbte_tuning;

/* Build options.  Channel selection (paper: scattering-channel paragraph
 * after Eq. 2: approximate energy conservation with the Gaussian delta and a
 * cutoff on |g|) and elastic mechanisms (paper, Discussion: other scattering
 * mechanisms, such as defects, on the same data structure).  Zero-initialised
 * options keep every channel and treat every mode as a phonon. */
typedef struct {
    double energy_nsigma;      /* > 0: keep channel (i, j, nu) only if
                                  min(|D + hw|, |D - hw|) < energy_nsigma * sigma,
                                  D = eps_i - eps_j, hw = hw(q = k_j - k_i, nu)
                                  (FP64); 0 = no energy cut                     */
    double g2_min;             /* keep a channel only if |g|^2 >= g2_min; 0 = all */
    uint32_t elastic_modes;    /* bit nu set: mode nu is an elastic mechanism (e-defect
                                  scattering on the same channel list): its hw must
                                  be 0 at every q, and the caller passes N = 0 for
                                  it, so that Eq. 2 reduces to the elastic golden
                                  rule K |g|^2 G(eps_i - eps_j) (f_j - f_i)         */
    int32_t statistics;        /* 0: Fermi (electrons, Eq. 2 as written).
                                  1: Bose: the same integral over the same channel
                                  list with the blocking factors (1 - f) replaced
                                  by the enhancement factors (1 + n), for
                                  phonon-phonon (three-phonon) scattering: states
                                  are phonon modes (energy in eps, occupation n in
                                  the f arguments), a channel (i, j, nu) couples
                                  modes i and j through the third phonon of branch
                                  nu at q = k_j - k_i, whose energy and occupation
                                  are hw and N (paper, Discussion: other scattering
                                  mechanisms on the same data structure).  Bose
                                  plans serve the collision integral, its reverse
                                  passes (collision_vjp, collision_vjp_nph), the
                                  RK4 steps and their adjoint; the other entry
                                  points return INVALID_ARGUMENT for them.        */
    int32_t reserved[2];       /* must be 0                                        */
} ephbte_build_opts;

/*
 * Build the device channel layout (paper: Optimized GPU algorithm, step 1,
 * "create the target layer": channels grouped by the collision-integral
 * element they feed, done once on the host).  Each channel is duplicated into
 * one entry per destination state, entries are sorted by destination and then
 * by (partner, mode), and the structure-of-arrays layout is copied to the
 * device once.  Fails with INVALID_ARGUMENT on: null pointers, indices out of
 * range, i == j, a pair not commensurate with the q grid, a channel of a
 * phonon mode whose energy is below 1e-6 eV in either orientation (its N
 * diverges; elastic modes excepted, whose hw must be 0),
 * duplicate (i, j, nu) channels, non-finite or negative hw/g2/eps, sigma or
 * n_q_norm <= 0, and options out of range.  Every channel is validated; the
 * selection of opts (NULL: none) then removes channels, and the plan computes
 * Eq. 2 over the ones kept: their |g|^2 gradients are 0, and ephbte_update_g2
 * does not re-run the selection.  Duplicates are detected among kept
 * channels.  OUT_OF_MEMORY if device memory runs out.  *out receives a plan
 * owned by the caller until ephbte_destroy.  Synchronous.
 */
ephbte_status ephbte_build_channels(const ephbte_problem *problem, const ephbte_build_opts *opts,
                                    ephbte_plan *out);

/*
 * Host-only view of the layout ephbte_build_channels would build with the
 * same options, for inspection and tests.  Runs the same validation,
 * selection and sort without touching a device.  Caller allocates: row_ptr
 * [S+1], entry_partner [2*n_channels], entry_mode [2*n_channels],
 * entry_channel [2*n_channels] (any may be NULL; the kept entries fill the
 * first row_ptr[S] slots).
 * Entry e of destination d (row_ptr[d] <= e < row_ptr[d+1]) has partner
 * entry_partner[e], mode entry_mode[e] and comes from caller channel
 * entry_channel[e].
 */
ephbte_status ephbte_layout_host(const ephbte_problem *problem, const ephbte_build_opts *opts,
                                 int64_t *row_ptr, int32_t *entry_partner, int8_t *entry_mode,
                                 int32_t *entry_channel);

/*
 * I[f] for B occupation vectors (Eq. 2; paper: Optimized GPU algorithm, steps
 * 2 and 3 fused into one pass over the channel list).
 * f:   device [B][ldf], plan dtype, 0 <= f <= 1 expected (not checked).
 * nph: device, plan dtype, phonon occupations N.  nph_per_batch == 0: one
 *      table [Nq][n_modes] shared by every vector (one (alpha, beta) per
 *      entry serves the whole batch).  nph_per_batch != 0: B tables
 *      [B][Nq][n_modes], vector b with its own bath; the vectors are then
 *      evaluated one after another, each a single-vector pass.
 * I:   device [B][ldi], plan dtype, written.  I must not alias f.
 * B >= 1; ldf, ldi >= S.
 * Reductions: with B = 1 and the single-copy layout every channel is read
 * once; the partner side is summed in 64-bit fixed point with integer
 * atomics (associative, so the result is bitwise reproducible), and so is the
 * row side over pair records in q order (pair_order 1); otherwise the row
 * side is summed in registers in a fixed order.  Other forms reduce each
 * destination's entries with no atomics.
 */
ephbte_status ephbte_collision_integral(ephbte_plan plan, int32_t batch, const void *f,
                                        int64_t ldf, const void *nph, int32_t nph_per_batch,
                                        void *I, int64_t ldi, void *stream);

/*
 * Allocation-free form of ephbte_collision_integral for callers that cannot
 * allocate device memory: code being captured into a HIP graph, serving loops
 * that must not call hipMalloc, harnesses that forbid it.  Same result as
 * ephbte_collision_integral with batch = 1 and one shared bath
 * (nph_per_batch = 0), from the same kernels.
 * f:   device [S], plan dtype.   nph: device [Nq][n_modes], plan dtype.
 * I:   device [S], plan dtype, written; must not overlap f.
 * Workspaces: the call allocates nothing (no hipMalloc, hipFree or allocating
 *   library routine).  Its {hw, N} table and partial sums live in a static
 *   device array of 32 MiB that the library holds on each GPU it runs on until
 *   the process ends.  A plan whose table and partials need more than that
 *   (2 x 8 B x Nq x n_modes plus 16 B per row chunk in FP64; the 50^3 q grid
 *   with 6 modes needs 12.4 MB) is rejected with EPHBTE_INVALID_ARGUMENT
 *   before any work is enqueued.
 * Concurrency: every call on one GPU shares that array and the plan's
 *   partner-side accumulator, and each call overwrites what the last one left
 *   there.  Calls on one plan are ordered like every other call; calls on
 *   different plans of one GPU that overlap in time (different streams, no
 *   ordering between them) race on the array and give wrong results.
 */
ephbte_status ephbte_collision_integral_noalloc(ephbte_plan plan, const void *f, const void *nph,
                                                void *I, void *stream);

/*
 * Reverse mode of Eq. 2: given gI = dL/dI (device [B][ldg]), writes
 * gf = dL/df (device [B][ldgf], plan dtype; NULL to skip) and
 * gg2 = dL/d|g|^2 summed over the batch (device FP64 [n_channels] in the
 * caller's channel order; NULL to skip).  accumulate_gg2 != 0 adds to gg2
 * instead of overwriting it.  nph and nph_per_batch as for
 * ephbte_collision_integral.  No atomics: dL/df is a per-destination
 * reduction, each dL/d|g|^2 is written by the channel's first entry.
 */
ephbte_status ephbte_collision_vjp(ephbte_plan plan, int32_t batch, const void *f,
                                   int64_t ldf, const void *nph, int32_t nph_per_batch,
                                   const void *gI, int64_t ldg, void *gf, int64_t ldgf,
                                   double *gg2, int32_t accumulate_gg2, void *stream);

/*
 * Phonon side of the same processes (coupled electron-phonon dynamics; the
 * paper cites this use of the method): dN/dt of every phonon (q, mode) from
 * the channel list.  Each entry (d, p, nu) adds, to the bin of phonon
 * (nu, q = k_p - k_d), its net emission Kp |g|^2 G(e_d - e_p + hw)
 * [(N + 1) f_p (1 - f_d) - N f_d (1 - f_p)], with Kp = 2 pi / (hbar N_k) and
 * N_k the full k-grid count.  Elastic mechanisms add nothing.
 * f: device [S] (one vector), plan dtype.  nph: device [Nq][n_modes].
 * dN: device [Nq][n_modes], plan dtype, written (1/fs).
 * Layout: at build the channels are grouped by the phonon pair {q, -q} they
 * exchange (one record per state pair with a |g|^2 slot per mode), so every
 * bin is the sum of one group's terms: one wave per chunk of records, partial
 * sums added in chunk order, no atomics (bitwise reproducible).  The first
 * call allocates the chunk partials.
 */
ephbte_status ephbte_phonon_rate(ephbte_plan plan, const void *f, const void *nph, void *dN,
                                 void *stream);

/*
 * Reverse of ephbte_phonon_rate: given gR = dL/d(dN/dt) (device [Nq][n_modes],
 * plan dtype), writes gf = dL/df (device [S], plan dtype), gnph = dL/dN
 * (device [Nq][n_modes], plan dtype) and adds (accumulate_gg2 != 0) or writes
 * gg2 = dL/d|g|^2 (device FP64 [n_channels], caller order); each output may be
 * NULL.  Derivatives of the rate's terms: the rate is quadratic in f and
 * affine in N and |g|^2 (elastic mechanisms contribute nothing).  dL/df is a
 * per-destination reduction over the destination layout; dL/dN and dL/d|g|^2
 * come from the records grouped by {q, -q}; no atomics.
 */
ephbte_status ephbte_phonon_rate_vjp(ephbte_plan plan, const void *f, const void *nph, const void *gR,
                                     void *gf, void *gnph, double *gg2, int32_t accumulate_gg2,
                                     void *stream);

/*
 * dL/dN of L = sum_d gI_d I_d (Eq. 2 at f and nph): gnph, device
 * [Nq][n_modes], plan dtype, overwritten.  Eq. 2 is affine in N: the summand
 * of destination d, partner p through (nu, q = k_p - k_d) has derivative
 * -K |g|^2 [G(e_d - e_p + hw) + G(e_d - e_p - hw)] (f_d - f_p) with respect to
 * N(q, nu) (K = 2 pi / (hbar N_q)); both orientations of every channel count,
 * elastic mechanisms included.  f, gI: device [S]; nph: device [Nq][n_modes].
 * Computed over the records grouped by {q, -q}, no atomics.
 */
ephbte_status ephbte_collision_vjp_nph(ephbte_plan plan, const void *f, const void *nph, const void *gI,
                                       void *gnph, void *stream);

/*
 * Coupled electron-phonon dynamics: advances f (device [S]) and the phonon
 * occupations nph (device [Nq][n_modes]) together, in place, by n_steps
 * classical RK4 steps of dt_fs: df/dt = I[f, N] (Eq. 2), dN/dt = the even
 * part in q of the rate of ephbte_phonon_rate.  Eq. 2 evaluates each
 * orientation of a channel with N at its own q, which is exact for N even in
 * q; the phonons of q and -q therefore evolve as a pair, which keeps an even
 * N even and, with hw even, moves the same energy.  Each stage packs the
 * stage's N and runs the electron pass (stage update fused in its epilogue)
 * and the phonon pass.  B = 1; no HIP graph; the field term of
 * ephbte_set_field is not applied here.  INVALID_ARGUMENT for NULL f or nph,
 * n_steps < 0, a non-finite dt_fs, or nph overlapping f; n_steps = 0 does
 * nothing.
 */
ephbte_status ephbte_rt_step_coupled(ephbte_plan plan, void *f, void *nph, double dt_fs,
                                     int32_t n_steps, void *stream);

/*
 * Reverse mode through n_steps coupled RK4 steps of ephbte_rt_step_coupled
 * from (f0, nph0): the exact discrete adjoint of the computed steps, for a
 * loss L(f_T, N_T) with gfT = dL/df_T (device [S]) and gNT = dL/dN_T (device
 * [Nq][n_modes]); either may be NULL (zero).  Writes gf0 = dL/df0 and
 * gN0 = dL/dnph0 (same shapes, plan dtype, nullable) and writes, or adds to
 * (accumulate_gg2 != 0), gg2 = dL/d|g|^2 (device FP64 [n_channels], caller
 * order, nullable).  Per stage (u, M) with adjoint (a, b) the transposed
 * Jacobian of the right-hand side (I[u, M], E R[u, M]), E the even part in q
 * (its own transpose), gives J_If^T a + J_Rf^T E b for f, J_IN^T a + J_RN^T E b
 * for N and J_Ig^T a + J_Rg^T E b for |g|^2.  (f, N) are checkpointed every
 * checkpoint_every steps and the stage inputs of a segment recomputed
 * (device memory: 4 checkpoint_every + 1 copies of (f, N)).  Not a step of
 * the paper (its code has no reverse mode).  INVALID_ARGUMENT for NULL f0 or
 * nph0, n_steps < 1, checkpoint_every < 1, a non-finite dt_fs, or gf0 / gN0
 * overlapping f0 / nph0.
 */
ephbte_status ephbte_rt_adjoint_coupled(ephbte_plan plan, const void *f0, const void *nph0, double dt_fs,
                                        int32_t n_steps, int32_t checkpoint_every, const void *gfT,
                                        const void *gNT, void *gf0, void *gN0, double *gg2,
                                        int32_t accumulate_gg2, void *stream);

/*
 * Field term of Eq. 1 for ephbte_rt_step and ephbte_rt_adjoint: they then
 * integrate df/dt = -(1/hbar) F . grad_k f + I[f].  The k derivative along grid
 * axis a is the central difference inside the state's band, periodic over the
 * k grid; a neighbour that is not in the state list (outside the energy
 * window) counts as empty.  rate[a] = F_a / (hbar dk_a) in 1/fs, with F the
 * force on the carrier (-e E for electrons) and dk_a the k-grid step, so the
 * term is -sum_a rate[a] (f(k + dk_a) - f(k - dk_a)) / 2.  All three 0 (the
 * default) switch it off; ephbte_collision_integral and ephbte_collision_vjp
 * never include it.  INVALID_ARGUMENT for a non-finite rate, or for a nonzero
 * one when some (k, band) is held by two states of the plan.  Drops cached
 * HIP graphs.  Synchronous.
 */
ephbte_status ephbte_set_field(ephbte_plan plan, const double rate[3]);

/*
 * Real-time BTE, df/dt = I[f] (Eq. 1; with the field term when
 * ephbte_set_field has set one): advances f
 * (device [B][ldf], in place) by n_steps classical RK4 steps of dt_fs.  The
 * stage updates are fused into the collision kernels (four launches per
 * step).  use_graph != 0 captures the step sequence in a HIP graph on the
 * first call and replays it (the graph is cached per (f, nph, dt, B, stream)).
 */
ephbte_status ephbte_rt_step(ephbte_plan plan, int32_t batch, void *f, int64_t ldf,
                             const void *nph, double dt_fs, int32_t n_steps, int32_t use_graph,
                             void *stream);

/*
 * Exact discrete adjoint of n_steps RK4 steps from f0 (device [S], B = 1):
 * given gfT = dL/df(T) (device [S]), writes gf0 = dL/df(0) (device [S], may be
 * NULL) and gg2 = dL/d|g|^2 (device FP64 [n_channels], caller order; may be
 * NULL; accumulate_gg2 != 0 adds).  Forward states are checkpointed every
 * checkpoint_every steps and recomputed segment by segment.
 */
ephbte_status ephbte_rt_adjoint(ephbte_plan plan, const void *f0, const void *nph,
                                double dt_fs, int32_t n_steps, int32_t checkpoint_every,
                                const void *gfT, void *gf0, double *gg2,
                                int32_t accumulate_gg2, void *stream);

/*
 * Iterative transport BTE (Eq. 1 at steady state with a weak field, I
 * linearised at f0): with J = dI/df at f0 = -diag(1/tau) + W,
 *   x_d = tau_d ( v_d df0/de + sum_p W_dp x_p ),  df0/de = -f0 (1-f0) / (k_B T),
 * iterated from the relaxation-time start x = tau v df0/de for the three field
 * directions, and the mobility mu_ab = -e sum_d v_a x_b / sum_d f0.
 * f0:  device [S] plan dtype, Fermi-Dirac occupations at temperature T_K.
 * vel: device [S][3] plan dtype (m/s).
 * nph: device [Nq][n_modes] plan dtype.
 * x_out: device [S][3] plan dtype (may be NULL), final iterate (fs m/s / eV).
 * mobility_cm2_per_Vs: host double[9], row-major mu_ab.
 * Stops when max|mu_new - mu_old| / max|mu_new| <= tol; NOT_CONVERGED after
 * max_iter iterations, or earlier when that relative change has not set a new
 * minimum for 5 iterations (the floor of the working precision, e.g. FP32
 * above a 1e-8 tolerance; ephbte_last_error says "stagnated"), with the last
 * iterate and mobility written in either case.  *iters and
 * *resid (host, may be NULL) receive the iteration count and last relative change.
 * Synchronises on `stream` once per iteration (9 scalars device to host).
 */
ephbte_status ephbte_iterate_transport(ephbte_plan plan, const void *f0, const void *vel,
                                       double T_K, const void *nph, double tol, int32_t max_iter,
                                       void *x_out, double *mobility_cm2_per_Vs, int32_t *iters,
                                       double *resid, void *stream);

/* Replace |g|^2 of every channel: g2 is device FP64 [n_channels] in the
 * caller's channel order (finite, >= 0 expected; not checked). */
ephbte_status ephbte_update_g2(ephbte_plan plan, const double *g2, void *stream);

/* Re-split the layout into workgroup chunks for the given tuning (no data is
 * re-sorted).  Synchronous. */
ephbte_status ephbte_set_tuning(ephbte_plan plan, const ephbte_tuning *tuning);

/* Time candidate tunings of the B-vector collision integral on this plan with
 * HIP events and keep the fastest; writes the chosen tuning to *chosen (may be
 * NULL).  For batch < 8 the candidates are chunk sizes x block sizes of the
 * single-vector kernel; for batch >= 8, partner sub-tile sizes of the batched
 * kernel.  Allocates and frees its own half-filled occupations.  Synchronous.
 * cache_path (may be NULL): a JSON file mapping a key (device architecture and
 * compute-unit count, dtype, states, entries, modes, q grid, single or
 * batched) to the tuning chosen for it.  An entry for this plan is applied
 * without timing; otherwise the tuning is timed and the file rewritten (via a
 * temporary file and a rename) with the new entry added.  INVALID_ARGUMENT if
 * the file holds something else (it is left alone) or cannot be written. */
ephbte_status ephbte_autotune(ephbte_plan plan, int32_t batch, ephbte_tuning *chosen,
                              const char *cache_path);

/* Launch timing of the forward pass's main kernel, for measurement (not a
 * step of the method): the single-copy kernel at B = 1, the per-row kernel for
 * B = 2 .. 7 (or layout 1) and the batched kernel for B >= 8.
 * mode 1: clears the record and starts it; every eager launch of that kernel
 *   on this plan is then bracketed by two HIP events recorded on its launch
 *   stream (launches under graph capture are not timed; at most 4096 launches
 *   per period are, later ones are not).
 * mode 0: stops it, waits for the recorded events, and returns the number of
 *   timed launches in *launches and their mean duration in ms in *mean_ms
 *   (0 when none); both host pointers may be NULL.
 * INVALID_ARGUMENT for another mode; HIP_ERROR if an event fails. */
ephbte_status ephbte_kernel_timing(ephbte_plan plan, int32_t mode, double *mean_ms, int64_t *launches);

/* Plan facts: out[0]=S, [1]=n_channels passed at build, [2]=entries,
 * [3]=chunks, [4]=dtype, [5]=device, [6]=device bytes held,
 * [7]=chunk_entries, [8]=block_threads, [9]=channels kept by the selection,
 * [10]=layout of the single-vector forward pass (ephbte_tuning.layout),
 * [11]=pair records of layout 3 (0: the plan has none). */
ephbte_status ephbte_plan_info(ephbte_plan plan, int64_t out[12]);

int64_t ephbte_plan_bytes(ephbte_plan plan);
void ephbte_destroy(ephbte_plan plan);
const char *ephbte_status_string(ephbte_status status);
const char *ephbte_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* EPHBTE_H */
