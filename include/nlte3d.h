/*
 * nlte3d.h -- C-ABI of the MI355X (gfx950) non-LTE 3D radiative-transfer library.
 *
 * The library solves the non-LTE problem of Bjorgen & Leenaarts (2017):
 * the transfer equation dI/dtau = S - I (Eq. 1) for every direction and frequency,
 * coupled to statistical equilibrium (Eq. 2) with the first rate equation replaced by
 * particle conservation (Eq. 3, right-hand side f = [n_tot, 0, ..., 0], Eq. 5).
 * The smoother is MALI with a diagonal approximate operator (Sect. 2.1, 3); it is
 * wrapped by nonlinear FAS multigrid V-cycles (Sect. 2.2, Eqs. 6-12) and full multigrid
 * (Sect. 2.3, Eqs. 13-14).  An atmosphere and a model atom go in; level populations,
 * line source functions and emergent intensities come out.
 *
 * Conventions for every entry point:
 *  - Units are CGS.  3D fields are C-ordered [z][y][x] with x fastest; z increases
 *    upward; x and y are periodic with uniform spacing.
 *  - The caller owns every buffer it passes.  *_create copies what it needs, so the
 *    caller may free descriptor memory when the call returns.  Output buffers are
 *    caller-allocated; a flag says whether a pointer is host or device memory.
 *  - Device work is enqueued on the context's HIP stream, except where an entry point
 *    says otherwise (graph replay and graph batches run on private streams ordered after
 *    the context's; served jobs run on streams of their own).  Calls that return host
 *    data synchronise that stream.  Calls on one context are serialised by a mutex.
 *  - Return value: 0 = success; negative = failure with nothing partially returned
 *    (nlte_last_error gives the message); positive = warning with the result valid.
 */
#ifndef NLTE3D_H
#define NLTE3D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status codes */
typedef int nlte_status;
#define NLTE_OK                 0
#define NLTE_E_INVALID         -1   /* bad argument, non-finite input, grid constraint */
#define NLTE_E_OOM             -2   /* device allocation failed or HBM budget exceeded */
#define NLTE_E_DEVICE          -3   /* HIP runtime error (text in nlte_last_error) */
#define NLTE_E_DIVERGED        -4   /* NaN/Inf or growing correction detected */
#define NLTE_W_NOT_CONVERGED    1   /* iteration cap reached; result readable */
#define NLTE_W_QUEUED           2   /* serving: request accepted, not yet admitted */

#define NLTE_MEM_HOST   0
#define NLTE_MEM_DEVICE 1

#define NLTE_MALI 0                 /* plain MALI (Jacobi ALI) iterations */
#define NLTE_FAS  1                 /* FAS V-cycles */
#define NLTE_FMG  2                 /* full multigrid followed by FAS V-cycles */

#define NLTE_SWEEP_AUTO        0    /* sweep kernel chosen per grid level */
#define NLTE_SWEEP_PLANE_STEP  1    /* plane state in HBM, one launch per plane step */

#define NLTE_FP64  0                /* formal solution in FP64 */
#define NLTE_MIXED 1                /* formal solution and accumulation in FP32; rate
                                       solves, normalisation, residual and coarse-grid
                                       right-hand side in FP64 */

#define NLTE_RESTRICT_FULL   0      /* full weighting, 27 points (Sect. 4.4) */
#define NLTE_RESTRICT_HALF   1      /* half weighting: the point 1/2, its six axis neighbours 1/12 each */
#define NLTE_RESTRICT_INJECT 2      /* injection: the fine value at the coarse point */

#define NLTE_INTERP_TRILINEAR 0     /* trilinear prolongation (Sect. 4.5) */
#define NLTE_INTERP_HERMITE   1     /* monotone cubic Hermite on the 4x4x4 coarse stencil */

#define NLTE_SC_BILINEAR 0          /* upwind I, S, chi by bilinear interpolation (Sect. 3) */
#define NLTE_SC_HERMITE  1          /* ... by monotone bicubic Hermite interpolation on 4x4 points */

#define NLTE_INIT_ZERO_RAD 0        /* zero-radiation populations (Sect. 4.11) */
#define NLTE_INIT_LTE      1        /* Saha-Boltzmann populations */
#define NLTE_INIT_USER     2        /* params.init_pops */

/* ---------------------------------------------------------------- handles */
typedef struct nlte_ctx nlte_ctx;
typedef struct nlte_atom nlte_atom;
typedef struct nlte_atmos nlte_atmos;
typedef int64_t nlte_job;

/* ---------------------------------------------------------------- descriptors */
typedef struct {
    double E;                  /* level energy above the atom's ground level, cm^-1 */
    double g;                  /* statistical weight */
    int stage;                 /* ionisation stage; a level of stage s+1 is a continuum */
} nlte_level_desc;

typedef struct {
    int lower, upper;          /* level indices, lower < upper energy */
    double A;                  /* Einstein A_ji, s^-1 */
    double gamma_rad;          /* radiative damping, s^-1 */
    double gamma_vdw;          /* van der Waals coefficient: Gamma += gamma_vdw n_H (T/5000)^0.3 */
    int nfreq;                 /* frequency points of this line */
    const double* q;           /* nfreq velocity offsets (cm/s), increasing; nu = nu0 (1 + q/c) */
} nlte_line_desc;

typedef struct {
    int lower, upper;          /* bound level and continuum level */
    double alpha0;             /* photo-ionisation cross-section at the edge, cm^2 (nu^-3 above) */
} nlte_cont_desc;

typedef struct {
    int lower, upper;
    double c_ul;               /* C_ul = n_e c_ul (T/T_ref)^beta; C_lu by detailed balance */
    double T_ref, beta;
} nlte_coll_desc;

typedef struct {
    int nlevel, nline, ncont, ncoll;
    double mass_amu;           /* atomic mass */
    double xi;                 /* microturbulence, cm/s */
    double epsilon;            /* > 0: two-level destruction probability (collisions ignored) */
    const nlte_level_desc* levels;
    const nlte_line_desc* lines;
    const nlte_cont_desc* continua;
    const nlte_coll_desc* collisions;
    int ncont_nu;              /* > 0: the continua are active transitions of the formal
                                  solution, swept at these frequencies (RH92 preconditioning
                                  of the overlapping continua, with the terms in every upper
                                  level's population: at most 4 distinct upper levels); every
                                  line frequency must then lie below every continuum edge,
                                  since the line sweeps carry no bound-free opacity
                                  (NLTE_E_INVALID otherwise), and jobs take the bilinear
                                  upwind interpolation (sc_interp); 0: fixed continua with
                                  photo-rates at J = B(T) */
    const double* cont_nu;     /* ncont_nu frequencies (Hz), increasing, containing every
                                  continuum edge; host memory, copied */
} nlte_atom_desc;

typedef struct {
    int nx, ny, nz;
    double dx, dy;             /* horizontal spacings, cm */
    const double* z;           /* nz heights (cm), strictly increasing; always host memory */
    const double *T, *ne, *nH, *ntot, *vx, *vy, *vz;   /* [nz][ny][nx] */
    const double* chi_c;       /* [nchi][nz][ny][nx] background opacity (cm^-1) per line, or NULL */
    int nchi;                  /* planes in chi_c (>= the atom's nline when chi_c is given) */
    int mem_kind;              /* NLTE_MEM_HOST or NLTE_MEM_DEVICE for the field arrays */
} nlte_atmos_desc;

typedef struct {
    int method;                /* NLTE_MALI / NLTE_FAS / NLTE_FMG */
    int precision;             /* NLTE_FP64 / NLTE_MIXED */
    int nlev;                  /* number of grids (1 for MALI) */
    int nu_fmg, nu0, nu1, nu2, nu3;   /* iteration counts (Sect. 2.2, 2.3, 4.12) */
    int init;                  /* NLTE_INIT_* */
    const double* init_pops;   /* NLTE_INIT_USER: [N][nz][ny][nx] host memory, the finest grid's
                                  populations (MALI and FAS; FMG starts from its coarsest
                                  grid and rejects them).  A FAS run resumed from the
                                  populations of an earlier one repeats that run's further
                                  cycles bit for bit when nu0 = 0 (nu0 > 0 applies to the
                                  first cycle of every run). */
    double tol_C;              /* stop when C <= tol_C (<= 0 disables) */
    double E_target;           /* stop when rho/(1-rho) C <= E_target, rho < 1 (<= 0 disables) */
    int max_iter;              /* cap on MALI iterations (MALI) or V-cycles (FAS/FMG) */
    double repair_frac;        /* negative-population repair fraction (0.1, Sect. 4.10) */
    int fallback_mali;         /* FAS/FMG: when the divergence guard fires (a non-finite cycle
                                  correction, or the growth test of diverge_cycles), restore
                                  the finest populations from the start of the failing cycle
                                  and continue with plain MALI iterations on the finest grid
                                  under the same stop rule (its C and rho from the MALI
                                  iterations alone), within max_iter further iterations;
                                  result.fallback = 1.  0: the run fails with
                                  NLTE_E_DIVERGED. */
    const double* top_I;       /* prescribed incoming intensity at the top [nf][ny][nx] or NULL */
    int dirs_per_block;        /* sweep directions per workgroup: 0 = autotune, else 3/6/12 where a
                                  level's frequency chunks (3/6/12 directions x 4/2/1 chunks
                                  per 12-wave block) and accumulator slots allow it, else
                                  autotuned there (results do not depend on it) */
    int timing;                /* 1: time each phase with HIP events on the context stream */
    int graph;                 /* 1: capture one V-cycle (FAS/FMG) or one MALI iteration as a
                                  HIP graph on a job-private stream and replay it; the first
                                  cycle (nu0) runs eagerly.  Phase timing is not available
                                  for replayed work. */
    int sweep_kernel;          /* NLTE_SWEEP_AUTO or NLTE_SWEEP_PLANE_STEP (the same kernel:
                                  plane state in HBM, one launch per plane step); other
                                  values are rejected with NLTE_E_INVALID */
    int restriction;           /* NLTE_RESTRICT_*: restriction of populations and residuals
                                  in FAS/FMG (Sect. 4.4); the paper's choice, and the
                                  zero default, is full weighting */
    int coarse_atmos;          /* NLTE_RESTRICT_*: how the coarse model atmospheres are made
                                  from the finer ones (Sect. 4.7); full weighting by default,
                                  injection the paper's alternative */
    int interpolation;         /* NLTE_INTERP_*: prolongation of corrections and of FMG full
                                  approximations (Sect. 4.5); trilinear by default, as in
                                  the paper's 3D runs */
    int sc_interp;             /* NLTE_SC_*: interpolation of the upwind intensity, source
                                  function and opacity in the short-characteristics formal
                                  solution (Sect. 3 names linear and Hermite-spline);
                                  bilinear by default.  Hermite runs the plane-step sweep
                                  with three directions per block and needs levels whose
                                  8-slot accumulators fit in 48 GiB; it applies to the
                                  emergent intensity too. */
    int diverge_cycles;        /* divergence guard of FAS/FMG (Sect. 4.10: cycles can diverge when
                                  coarse grids produce many negative populations): the run
                                  diverges when the cycle correction C grows, C_i >
                                  diverge_growth C_{i-1} with C_i > 1e-3, in this many
                                  consecutive cycles; 0 = 3, < 0 = off (a non-finite C
                                  always counts) */
    double diverge_growth;     /* growth factor of that test; 0 = 1 */
} nlte_params;

typedef struct {
    int status;
    int iterations;            /* finest-level MALI iterations (MALI) */
    int cycles;                /* V-cycles at the finest level */
    double C;                  /* last max relative change (Eq. 16) */
    double rho;                /* last C_i / C_{i-1} */
    double E_est;              /* rho / (1 - rho) C (Eq. 18) */
    long long repairs;         /* negative-population repairs */
    long long formal_solutions[8];   /* per level, index 0 = coarsest */
    double fine_fs_equiv;      /* work in finest-grid formal solutions (Sect. 4.9 cost units) */
    double updates;            /* voxel x direction x frequency updates performed */
    double ms_total, ms_setup, ms_sweep, ms_rates, ms_transfer;   /* phase times need params.timing */
    long long sweep_launches;  /* plane-step sweep kernel launches (formal solutions x planes) */
    int dirs_per_block;        /* sweep block shape used on the finest level (3, 6 or 12; 0 if none ran) */
    int sweep_kernel;          /* NLTE_SWEEP_PLANE_STEP */
    int fallback;              /* 1: FAS/FMG diverged and the run continued as plain MALI
                                  (params.fallback_mali); iterations counts those MALI
                                  iterations and cycles the cycles before it */
} nlte_result;

/* ---------------------------------------------------------------- lifecycle */
/* Create a context on HIP device `device` that enqueues on `hip_stream` (a hipStream_t,
 * NULL = the device's null stream).  `hbm_budget` bounds the bytes the context may
 * allocate (0 = 90 % of free device memory).  If the environment variable
 * NLTE3D_TUNE_CACHE names a file, the sweep autotuner's choices for this device's
 * architecture are read from it (a flat JSON object; unreadable or malformed files count
 * as empty) and every new choice is merged into it. */
nlte_status nlte_ctx_create(int device, void* hip_stream, size_t hbm_budget, nlte_ctx** out);
void nlte_ctx_destroy(nlte_ctx* ctx);
/* Message of the last failing call on ctx (empty string if none); owned by ctx. */
const char* nlte_last_error(const nlte_ctx* ctx);
/* Library version string. */
const char* nlte_version(void);

/* Copy a model atom (Sect. 3.2).  Fails with NLTE_E_INVALID for inconsistent indices,
 * non-positive g/A/mass, fewer than 2 frequencies or non-increasing q. */
nlte_status nlte_atom_create(nlte_ctx* ctx, const nlte_atom_desc* desc, nlte_atom** out);
void nlte_atom_destroy(nlte_ctx* ctx, nlte_atom* atom);

/* Copy a model atmosphere (Sect. 3.1) to the device.  Validation: finite values,
 * T > 0, densities >= 0, n_tot > 0, z strictly increasing. */
nlte_status nlte_atmos_create(nlte_ctx* ctx, const nlte_atmos_desc* desc, nlte_atmos** out);
void nlte_atmos_destroy(nlte_ctx* ctx, nlte_atmos* atmos);

/* ---------------------------------------------------------------- solving */
/* Build the grid hierarchy (Sect. 4.1, 4.2: nx, ny and nz-1 divisible by 2^(nlev-1),
 * else NLTE_E_INVALID), the coarse atmospheres by full weighting (Sect. 4.7), the
 * local physics of every level and the initial populations.  The atom and atmosphere
 * may be destroyed afterwards.  The job keeps its populations resident on the device. */
nlte_status nlte_job_create(nlte_ctx* ctx, const nlte_atmos* atmos, const nlte_atom* atom,
                            const nlte_params* params, nlte_job* job);
/* Run the method chosen in params to the stop rule (or max_iter). */
nlte_status nlte_job_run(nlte_ctx* ctx, nlte_job job, nlte_result* result);
/* job_create + job_run. */
nlte_status nlte_solve(nlte_ctx* ctx, const nlte_atmos* atmos, const nlte_atom* atom,
                       const nlte_params* params, nlte_result* result, nlte_job* job);
/* Free the job's device state. */
nlte_status nlte_release(nlte_ctx* ctx, nlte_job job);
/* Run several created jobs to their stop rules together.  Small grids underfill the GPU
 * (Sect. 4.9: coarse grids cost more than their share), so every plane step of the jobs'
 * formal solutions is one launch per class of frequency chunks over a device work list of
 * (job, plane tile, line, direction group) items; the rest runs per job, on the context's
 * stream.  The jobs go through the same method schedule in lockstep and each leaves the
 * batch when its own stop rule, iteration cap or divergence guard ends its run.  Each job's
 * populations and history are bit for bit those of nlte_job_run on it alone.  The jobs must
 * share precision, method, number of grids and iteration counts (nu_fmg, nu0..nu3), sweep
 * with the plane-step kernel and bilinear upwind interpolation in one frequency pass, have
 * no active continua, and all or none ask for graph replay (params.graph; else
 * NLTE_E_INVALID before any work); sizes, atoms and stop rules may differ.  With graph
 * replay the batch runs on a private stream that follows the context's: each repeated step
 * of a job set (a MALI iteration, a cycle after the first) runs eagerly once, is captured
 * as a HIP graph the next time and replayed after that.  results[j] (njobs entries) gets
 * job j's result, with ms_sweep the batch's sweep time (eager steps only).  Returns the most severe warning of the jobs, or the
 * error of the first job that failed (the other results stay valid). */
nlte_status nlte_batch_run(nlte_ctx* ctx, int njobs, const nlte_job* jobs, nlte_result* results);

/* ---------------------------------------------------------------- outputs */
/* Populations of grid `level` (0 = coarsest, nlev-1 = finest) as [N][nz][ny][nx] FP64. */
nlte_status nlte_get_populations(nlte_ctx* ctx, nlte_job job, int level, double* dst, int dst_mem);
/* Overwrite the populations of grid `level` (same layout). */
nlte_status nlte_set_populations(nlte_ctx* ctx, nlte_job job, int level, const double* src, int src_mem);
/* Line source functions S_l = n_j A_ji / (n_i B_ij - n_j B_ji) on the finest grid,
 * [nline][nz][ny][nx] FP64; NaN where the denominator is <= 0. */
nlte_status nlte_get_source_function(nlte_ctx* ctx, nlte_job job, double* dst, int dst_mem);
/* Emergent intensity at the top plane for `ndir` upward directions mu[ndir][3]
 * (normalised internally), after a formal solution at the finest populations
 * (Sect. 5, Fig. 10 uses mu_z = 1).  dst: [ndir][nf][ny][nx] FP32, nf = total
 * frequencies of all lines in atom order. */
nlte_status nlte_emergent_intensity(nlte_ctx* ctx, nlte_job job, int ndir, const double* mu,
                                    float* dst, int dst_mem);
/* Emergent intensity at the continuum frequencies of an atom with active continua
 * (nlte_atom_desc.ncont_nu > 0; NLTE_E_INVALID otherwise), for `ndir` upward directions
 * mu[ndir][3] (normalised internally): an upward formal solution in FP64 from the finest
 * populations with the continua's opacity and source function, B_nu(T) at the lower
 * boundary and bilinear upwind interpolation (the emergent spectrum of Sect. 5, Fig. 10,
 * at the continuum frequencies).  dst: [ndir][ncont_nu][ny][nx] FP32, frequencies in the
 * order of cont_nu; dst_mem says whether dst is host or device memory. */
nlte_status nlte_emergent_continuum_intensity(nlte_ctx* ctx, nlte_job job, int ndir, const double* mu,
                                              float* dst, int dst_mem);
/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): nlte_emergent_intensity with the
 * output in device memory (dst: [ndir][nf][ny][nx] FP32, host memory is rejected with
 * NLTE_E_INVALID), computed by the same kernels, bit for bit the same values, with no
 * device allocation or free.  The upward formal solution's plane state lives in a 48 MiB
 * static device array that the library keeps on every GPU it runs on until the process
 * ends; frequencies are processed in chunks of 1048576 / (nx ny) (at least one: planes
 * of more than 1048576 points are rejected with NLTE_E_INVALID).  Every call on one GPU
 * shares that array, which keeps the last call's contents (each call writes every state
 * element before reading it): calls that overlap on one GPU, from several contexts or
 * threads, race. */
nlte_status nlte_emergent_intensity_noalloc(nlte_ctx* ctx, nlte_job job, int ndir, const double* mu, float* dst);
/* The job's work so far, including stage-hook calls: formal solutions per level, finest-grid
 * formal-solution equivalents, updates, sweep launches and block shape, repairs, the last C,
 * and (with params.timing) the phase times measured with HIP events on the job's stream;
 * status, iterations, cycles, rho and E_est are those of the last nlte_job_run (0 before). */
nlte_status nlte_job_stats(nlte_ctx* ctx, nlte_job job, nlte_result* out);
/* Convergence history: up to `cap` values of C per MALI iteration (MALI) or per cycle
 * (FAS/FMG; after a fallback to MALI the MALI iterations follow the cycles).  Returns the
 * number of values held, or -1 for an unknown job. */
int nlte_history(nlte_ctx* ctx, nlte_job job, double* C, int cap);

/* ---------------------------------------------------------------- stage hooks
 * Single steps of the method on one grid level, for parity tests.  The job's
 * precision decides the element type of jeff/oml: FP64 -> double, MIXED -> float. */
/* Formal solution at the level's current populations (Sect. 3): per line and voxel
 * Jeff = sum w phi~ (I_u e + Psi_u S_u + Psi_o eta_c/chi) and
 * 1-L* = sum w phi~ ((1-Psi_o) + Psi_o chi_c/chi); [nline][nz][ny][nx]. */
nlte_status nlte_formal_solution(nlte_ctx* ctx, nlte_job job, int level, void* jeff, void* oml, int dst_mem);
/* `iters` MALI iterations on `level` with that level's right-hand side; *C_out gets C
 * of the last iteration (may be NULL). */
nlte_status nlte_mali(nlte_ctx* ctx, nlte_job job, int level, int iters, double* C_out);
/* One rate solve on `level` from given radiation (Eqs. 3, 5 and the preconditioned rates
 * of Sect. 3): jeff = J-bar^eff and oml = 1 - Lambda-bar* per line and voxel,
 * [nline][nz][ny][nx] in the job's precision (FP64 -> double, MIXED -> float), host or device
 * memory per src_mem (NLTE_MEM_*), take the place of the formal solution's sums.  The
 * level's populations are overwritten with the solution of the rate equations (row 0
 * replaced by conservation with the level's right-hand side, rescaled so that the
 * populations sum to it); *C_out (may be NULL) gets the maximum relative change.  Atoms
 * with active continua are rejected (NLTE_E_INVALID): their continuum sums come from the
 * formal solution only. */
nlte_status nlte_rate_solve(nlte_ctx* ctx, nlte_job job, int level, const void* jeff, const void* oml, int src_mem,
                            double* C_out);
/* Residual r = f - W(n) with an extra formal solution (Eq. 7), [N][nz][ny][nx] FP64. */
nlte_status nlte_residual(nlte_ctx* ctx, nlte_job job, int level, double* dst, int dst_mem);
/* One V-cycle on levels `level`..0 (Sect. 2.2); `first` applies nu0 at the top.
 * *repairs (may be NULL) gets the job's count of negative-population repairs so far
 * (Sect. 4.10: entries where the corrected population n_old (1 + I e) was <= 0 and
 * repair_frac * n_old was taken instead). */
nlte_status nlte_vcycle(nlte_ctx* ctx, nlte_job job, int level, int first, long long* repairs);
/* Full-weighting restriction (Sect. 4.4) of q fields [q][nz][ny][nx] (FP64) from grid
 * `level` to grid `level-1`; src and dst are device pointers (host memory is rejected with
 * NLTE_E_INVALID). */
nlte_status nlte_restrict(nlte_ctx* ctx, nlte_job job, int level, int nq, const double* src, double* dst);
/* Trilinear prolongation (Sect. 4.5) of q fields from grid `level-1` to `level` (device
 * pointers, as for the restriction). */
nlte_status nlte_prolong(nlte_ctx* ctx, nlte_job job, int level, int nq, const double* src, double* dst);
/* The Voigt function H(a, u) = Re w(u + i a) that the sweeps use for the line profile
 * (Sect. 3; phi = H / (sqrt(pi) dnu_D)), at n points of the device arrays a and u (FP64,
 * a >= 0), written to the device array H.  precision NLTE_FP64: the FP64 evaluation;
 * NLTE_MIXED: the FP32 evaluation (inputs rounded to FP32 first, the result widened).
 * Synchronises the context's stream; n = 0 does nothing; host memory is rejected with
 * NLTE_E_INVALID. */
nlte_status nlte_voigt(nlte_ctx* ctx, int precision, int n, const double* a, const double* u, double* H);

/* ---------------------------------------------------------------- serving
 * Continuous batching of many solves on one context.  nlte_submit queues a solve and
 * returns NLTE_W_QUEUED at once; worker threads admit queued solves in FIFO order as
 * soon as their device footprint fits the unreserved part of the HBM budget (the memory
 * of finished jobs counts until nlte_release; a job larger than the whole budget is
 * rejected at submission), build and run each on its own HIP stream, so the
 * kernels of concurrent solves overlap on the device, and keep the populations resident
 * until nlte_release.  The caller keeps `atmos` and `atom` alive until the job leaves
 * the queue (state >= NLTE_JOB_RUNNING has been observed) and passes no host arrays in
 * `params` (init_pops, top_I must be NULL).  Results are read with the output calls
 * above once the job is done.  Each solve is computed exactly as it would be alone. */
#define NLTE_JOB_QUEUED  0
#define NLTE_JOB_RUNNING 1
#define NLTE_JOB_DONE    2
#define NLTE_JOB_FAILED  3

typedef struct {
    int state;                 /* NLTE_JOB_* */
    int status;                /* final status of a finished job */
    double t_submit, t_admit, t_done;   /* seconds on a monotonic clock */
    size_t footprint;          /* device bytes reserved at admission */
    int batch;                 /* serving batch the job ran in (nlte_serve_batching), 0 if alone */
    nlte_result result;        /* valid when state == NLTE_JOB_DONE */
    char error[256];           /* message of a failed job */
} nlte_job_info_t;

/* Start up to `max_running` worker threads (1..16): the number of concurrent solves. */
nlte_status nlte_serve_config(nlte_ctx* ctx, int max_running);
/* Continuous batching of served jobs (1..64; 1, the default, runs each job alone): a
 * worker runs the job it admits together with queued jobs that can share its batch (as in
 * nlte_batch_run: one precision, method, number of grids and iteration counts, plane-step
 * bilinear sweeps, no active continua, the same graph setting), up to batch_max at a time, in queue
 * order as their footprints fit the budget; between cycles (MALI: iterations) it admits
 * more such jobs into the running batch, and each job is published as soon as its own run
 * ends.  Only grids too small to fill the device alone are batched: a batch's summed
 * finest plane-step work (nx * ny * 24 directions * frequencies) stays within that of a
 * 64 x 64 plane of 505 frequencies, and its jobs' finest formal solutions are within a
 * factor 4 of its first job's (the batch advances them in lockstep).  Other jobs run alone
 * on their own streams.  Results are bit for bit those of the same jobs alone. */
nlte_status nlte_serve_batching(nlte_ctx* ctx, int batch_max);
/* Device bytes a job with these inputs will allocate (its admission footprint). */
nlte_status nlte_estimate_footprint(nlte_ctx* ctx, const nlte_atmos* atmos, const nlte_atom* atom,
                                    const nlte_params* params, size_t* bytes);
/* Queue a solve; returns NLTE_W_QUEUED with *job set, or a negative error. */
nlte_status nlte_submit(nlte_ctx* ctx, const nlte_atmos* atmos, const nlte_atom* atom,
                        const nlte_params* params, nlte_job* job);
/* Current NLTE_JOB_* state of a submitted job. */
nlte_status nlte_poll(nlte_ctx* ctx, nlte_job job, int* state);
/* Block until the job finishes (its final status) or `timeout_ms` passes (NLTE_W_QUEUED;
 * a negative timeout waits forever). */
nlte_status nlte_wait(nlte_ctx* ctx, nlte_job job, int timeout_ms);
/* State, timestamps, footprint and result of a submitted job. */
nlte_status nlte_job_info(nlte_ctx* ctx, nlte_job job, nlte_job_info_t* info);

#ifdef __cplusplus
}
#endif
#endif /* NLTE3D_H */
