/*
 * nbody.h -- C ABI of the MI355X (gfx950) direct-summation N-body library (libnbody.so).
 *
 * The operations are those of NBSymple (Capuzzo-Dolcetta, Mastrobuono-Battisti & Maschietti,
 * New Astronomy):
 *   - the softened pairwise gravitational acceleration of Sect. 2, Eq. 5, and the softened pair
 *     potential of Eq. 4 summed over j != i;
 *   - the external field term of Eq. 3 (an analytic bulge + disk + halo galaxy, Sect. 3);
 *   - the kick and drift stages of the 2nd-order leapfrog and of the 6th-order symplectic
 *     composition of Sect. 3.1;
 *   - the energy, momentum, angular momentum and torque diagnostics of Sect. 5.1, Eqs. 8-10, and
 *     the mass-weighted sum of the internal accelerations, which the antisymmetry of the pair
 *     forces of Eq. 2 makes zero (a check of momentum conservation, Sect. 5.1).
 *
 * Data model
 *   A "system" is a ragged batch of B >= 1 independent clusters (they never interact).  Cluster b
 *   owns particles [offsets[b], offsets[b+1]) of every particle array.  All particle arrays are
 *   DEVICE pointers to contiguous row-major float64 data: pos, vel, acc are (Ntot, 3), mass and
 *   pot are (Ntot).  The caller owns them, the workspace and the context; the library never
 *   allocates device memory on a call path and never synchronises the stream (a call may wait on
 *   the host for the table upload of the fourth-previous call to finish, to reuse its pinned
 *   staging buffer).
 *
 * Units and signs
 *   a_i = G sum_{j != i} m_j d_ij / (|d_ij|^2 + eps_b^2)^{3/2} + a_ext(x_i),  d_ij = x_j - x_i
 *   pot_i = -G sum_{j != i} m_j / sqrt(|d_ij|^2 + eps_b^2)   (negative for bound systems)
 *   When eps_b > 0 the j = i term is exactly zero and the kernels may include it; when
 *   eps_b = 0 it is excluded explicitly.  The pair sum is evaluated in full (N^2 terms per
 *   cluster, no use of Newton's third law), as the paper does in Sect. 4.2.
 *
 * Precision modes (nbody_system.prec)
 *   NB_FP32    pure single precision: pairs, accumulation and state updates in FP32; every state
 *              value the library writes is an FP32 value stored in the float64 arrays.
 *   NB_FP32C   FP32 pair arithmetic on coordinates taken relative to each cluster's centre of
 *              mass (computed in FP64); per-tile FP32 partial sums folded into FP64; FP64 state.
 *   NB_FP32DS  as NB_FP32C, but every coordinate is held as a double-single pair (hi + lo FP32)
 *              and the coordinate difference of each pair is formed from both parts, the
 *              precision-recovery scheme of Sect. 5.2.
 *   NB_FP64    all FP64.
 *   NB_FP32DL  the accuracy of NB_FP32DS at close to the cost of NB_FP32C: each evaluation sorts
 *              every cluster's particles along a Hilbert curve of their FP64 positions; each pair
 *              work item takes coordinates relative to the centre of its own i-particles' bounding
 *              box; a j-tile all of whose sources lie at least 3/4 of the box diagonal from that
 *              centre is computed in FP32 on those local coordinates (coordinate-difference error
 *              at most 1.5 x 2^-22 relative), any other in double-single as NB_FP32DS.  Sums
 *              folded into FP64 per tile as in NB_FP32C.
 *
 * Errors
 *   Every function returns NB_OK (0) or a negative status.  All argument checks run on the host
 *   before any HIP call, so a rejected call launches nothing and leaves every buffer untouched.
 *   HIP runtime failures return NB_ERR_HIP.  nbody_last_error() returns a thread-local message
 *   for the last failing call on the calling thread.
 *
 * Threading
 *   A context may be used from one host thread at a time.  Calls that share a workspace must be
 *   ordered on one stream; calls on different streams need different workspaces.
 */
#ifndef NBODY_H
#define NBODY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nbody_ctx nbody_ctx;

enum {
  NB_OK = 0,
  NB_ERR_ARG = -1,         /* invalid argument; nothing was launched */
  NB_ERR_HIP = -2,         /* a HIP runtime call failed */
  NB_ERR_NOMEM = -3,       /* host-side allocation failed, or workspace too small */
  NB_ERR_UNSUPPORTED = -4, /* valid request the library does not implement */
  NB_ERR_NONFINITE = -5    /* not returned: nbody_energy is asynchronous and cannot see its own
                              sums, so it reports non-finite ones in its output (flag out[b][19]) */
};

enum { NB_FP32 = 0, NB_FP32C = 1, NB_FP32DS = 2, NB_FP64 = 3, NB_FP32DL = 4 };

/* External galaxy (Eq. 3, F_ext).  model NB_GALAXY_HERNQUIST_LOG (0), G-scaled except the halo:
 *   Hernquist bulge      Phi_b  = -G Mb / (r + ab)
 *   Miyamoto-Nagai disk  Phi_d  = -G Md / sqrt(R^2 + (ad + sqrt(z^2 + bd^2))^2)
 *   logarithmic halo     Phi_h  = vh^2 / 2 ln(r^2 + dh^2)
 * model NB_GALAXY_ALLEN_SANTILLAN (1), the Galaxy of Allen & Santillan (1991) that Sect. 3 names
 * (spherical bulge and halo, axisymmetric disk), all G-scaled; vh and dh are not used:
 *   bulge                Phi_b  = -G Mb / sqrt(r^2 + ab^2)
 *   Miyamoto-Nagai disk  as in model 0
 *   halo                 mass inside r  M(r) = Mh (r/ah)^2.02 / (1 + (r/ah)^1.02) for r < rcut, and
 *                        M(rcut) beyond; Phi_h = -G M(r)/r - G Mh/(1.02 ah) [H(rcut) - H(r)] with
 *                        H(s) = ln(1 + (s/ah)^1.02) - 1.02 / (1 + (s/ah)^1.02) for r < rcut, and
 *                        -G M(rcut)/r beyond (its published parameters, in kpc and 2.32e7 solar
 *                        masses with G = 1: Mb 606, ab 0.3873, Md 3690, ad 5.3178, bd 0.25,
 *                        Mh 4615, ah 12, rcut 100)
 * both models:
 *   central black hole   Phi_bh = -G Mbh / sqrt(r^2 + ebh^2)   (Sect. 6.2: a massive point fixed
 *                        at the galaxy centre; Mbh = 0 leaves it out)
 * with R^2 = x^2 + y^2 and r^2 = R^2 + z^2; a_ext = -grad(Phi_b + Phi_d + Phi_h + Phi_bh).
 * Mbh > 0 with ebh = 0 is singular at the origin (a particle exactly there gets a non-finite
 * acceleration, which the energy diagnostics flag).  Mh, ah and rcut are read by model 1 only. */
enum { NB_GALAXY_HERNQUIST_LOG = 0, NB_GALAXY_ALLEN_SANTILLAN = 1 };
typedef struct {
  double Mb, ab, Md, ad, bd, vh, dh;
  double Mbh, ebh;
  int32_t model;          /* NB_GALAXY_HERNQUIST_LOG or NB_GALAXY_ALLEN_SANTILLAN */
  double Mh, ah, rcut;    /* model 1's halo */
} nbody_galaxy;

/* A ragged batch of clusters.  All pointers are HOST pointers read during the call only. */
typedef struct {
  int32_t nclusters;      /* B >= 1 */
  const int64_t* offsets; /* [B+1], offsets[0] = 0, strictly increasing (every cluster >= 1) */
  double G;               /* gravitational constant, > 0 */
  const double* eps;      /* [B] softening lengths, each >= 0 and finite */
  const uint8_t* field;   /* [B] nonzero = add the galaxy field to that cluster; NULL = none */
  nbody_galaxy galaxy;    /* used by clusters whose field flag is set */
  int32_t prec;           /* NB_FP32 .. NB_FP32DL */
} nbody_system;

/* Create a context bound to HIP device `device` (>= 0).  The context caches launch plans and
 * tile choices; it owns a small pinned host staging area (NB_NOALLOC_TABLE_BYTES for the
 * no-allocation entry point, plus a ring that grows with the tables of the other calls) and never
 * allocates device memory.  It also looks up the device's copy of the static scratch of
 * nbody_accel_noalloc (the first context on a device loads the library's code objects there).
 * Returns NB_ERR_ARG for a bad device or NULL out, NB_ERR_HIP if the device cannot be used. */
int nbody_create(int device, nbody_ctx** out);

/* Destroy a context (NULL is allowed).  Waits for the staging copies it issued. */
void nbody_destroy(nbody_ctx* ctx);

/* Bytes of device workspace the calls below need for `sys` (0 if `sys` is invalid; then
 * nbody_last_error() says why): 32 bytes per particle, plus 32 bytes per particle and j-range
 * for clusters whose sums are split into several source ranges (a cluster of N particles uses
 * about 2^22/N ranges, a power of two of at most 8 (16 from 2^15 particles on) with at least 128
 * sources each, so clusters of 256..2^21 particles are split; an unsplit cluster in the
 * NB_GALAXY_ALLEN_SANTILLAN field takes one such range too, since a separate pass finishes it),
 * plus 48 bytes per particle, 4 KiB per 2048 particles and 4 KiB per cluster for the sort of
 * NB_FP32DL, and for its per-item frames and far-tile bits 32 bytes per
 * 64 particles and range plus N_b^2 / 2^15 bytes per cluster, plus O(B + N/64) bookkeeping.  The
 * workspace must be 256-byte aligned;
 * its contents are the library's between calls (the caller must not modify it while calls using
 * it are in flight). */
size_t nbody_workspace_bytes(const nbody_ctx* ctx, const nbody_system* sys);

/* An upper bound of nbody_workspace_bytes over every system of at most max_particles particles
 * in at most max_clusters clusters (any sizes, modes, softenings): what a caller that changes its
 * batch over time (the server) allocates once.  0 on invalid arguments. */
size_t nbody_workspace_bytes_max(int64_t max_particles, int32_t max_clusters);

/* Accelerations (Eq. 5 + external field of Eq. 3) of every particle of every cluster:
 *   acc[i] = a_i as defined above;  pot[i] = pair potential as defined above (pot may be NULL).
 * pos, mass: device, read.  acc, pot: device, written.  ws: device workspace of ws_bytes bytes.
 * stream: a hipStream_t (NULL = the default stream).  Asynchronous. */
int nbody_accel(nbody_ctx* ctx, const nbody_system* sys, const double* pos, const double* mass,
                double* acc, double* pot, void* ws, size_t ws_bytes, void* stream);

/* nbody_accel without a caller workspace, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid allocation).  The workspace
 * is a static device array of NB_NOALLOC_SCRATCH_BYTES inside the library, one per GPU, held from
 * the library's first use on that GPU until the process ends; the tables go up through a pinned
 * staging buffer of NB_NOALLOC_TABLE_BYTES that nbody_create allocated.  The call itself allocates
 * nothing (no hipMalloc, hipFree or pinned allocation).  Same arguments, results and errors as
 * nbody_accel, and bitwise the same accelerations and potentials.  Limits: a system whose
 * nbody_workspace_bytes exceeds NB_NOALLOC_SCRATCH_BYTES (a single cluster of more than about 8.1
 * million particles, 1.4 million in NB_FP32DL) or whose tables exceed NB_NOALLOC_TABLE_BYTES (more
 * than about 39,000 clusters) returns NB_ERR_ARG; these two checks run first and need
 * neither a context nor a GPU.  Every call on one GPU shares that GPU's scratch, which keeps the
 * last call's contents (the per-call counters are cleared by the call's own table upload): calls
 * that overlap on one GPU (several streams, threads or contexts at once) race and give wrong
 * results, so order them on one stream.  Asynchronous. */
#define NB_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
#define NB_NOALLOC_TABLE_BYTES ((size_t)4 << 20)
int nbody_accel_noalloc(nbody_ctx* ctx, const nbody_system* sys, const double* pos, const double* mass,
                        double* acc, double* pot, void* stream);

/* One integrator stage for every cluster b, with per-cluster coefficients (time step folded in):
 *   vel += kick_pre[b] * acc;  pos += drift[b] * vel;  acc = A(pos);  vel += kick_post[b] * acc
 * where A is the acceleration of nbody_accel.  This is the kick-drift-kick stage of which both
 * integrators of Sect. 3.1 are made: the leapfrog is one stage with (dt/2, dt, dt/2); the
 * 6th-order composition is seven stages with the weights of nbody_sym6_coefficients.  kick_pre, drift, kick_post: HOST arrays [B],
 * finite.  acc must hold A(pos) on entry (first-same-as-last).  This is the unit the
 * continuous-batching server advances each job by; the step functions below are sequences of it.
 * Asynchronous. */
int nbody_substep(nbody_ctx* ctx, const nbody_system* sys, double* pos, double* vel, const double* mass,
                  double* acc, const double* kick_pre, const double* drift, const double* kick_post,
                  void* ws, size_t ws_bytes, void* stream);

/* nrounds (1..64) consecutive nbody_substep rounds (Sect. 3.1 stages, as above) in one call: coef is
 * a HOST array
 * [nrounds][B][3] of (kick_pre, drift, kick_post) per round and cluster, all finite.  Round r
 * performs exactly what nbody_substep would with coef[r].  One table upload for all rounds; lets a
 * batching caller chain rounds while the set of clusters does not change.  Asynchronous. */
int nbody_substeps(nbody_ctx* ctx, const nbody_system* sys, double* pos, double* vel, const double* mass,
                   double* acc, const double* coef, int32_t nrounds, void* ws, size_t ws_bytes, void* stream);

/* nsteps (>= 0) steps of the 2nd-order leapfrog (Sect. 3.1) in kick-drift-kick form, step dt
 * (finite, any sign: a negative dt integrates backwards):
 *   vel += dt/2 acc;  pos += dt vel;  acc = A(pos);  vel += dt/2 acc
 * acc: on entry A(pos) (obtain it once with nbody_accel), on return A(pos_final).
 * One force evaluation per step.  Asynchronous. */
int nbody_step_leapfrog(nbody_ctx* ctx, const nbody_system* sys, double* pos, double* vel, const double* mass,
                        double* acc, double dt, int32_t nsteps, void* ws, size_t ws_bytes, void* stream);

/* nsteps steps of the 6th-order symplectic integrator of Sect. 3.1: the symmetric composition
 * S2(w3 h) S2(w2 h) S2(w1 h) S2(w0 h) S2(w1 h) S2(w2 h) S2(w3 h) of kick-drift-kick leapfrogs
 * (Yoshida 1990, solution A: w1 = -1.17767998417887, w2 = 0.235573213359357,
 * w3 = 0.784513610477560, w0 = 1 - 2(w1 + w2 + w3)), with the touching half-kicks inside one step
 * merged: 7 drifts, 8 kicks, 7 force evaluations per step.  Same arguments as the leapfrog. */
int nbody_step_sym6(nbody_ctx* ctx, const nbody_system* sys, double* pos, double* vel, const double* mass,
                    double* acc, double dt, int32_t nsteps, void* ws, size_t ws_bytes, void* stream);

/* The 7 drift and 8 kick weights of the 6th-order composition above (drift7[k] = w of stage k,
 * kick8[0] = w3/2, kick8[k] = (w_{k-1} + w_k)/2, kick8[7] = w3/2), as nbody_step_sym6 uses them;
 * host arrays.  Lets a caller drive the same integrator one stage at a time with nbody_substep. */
int nbody_sym6_coefficients(double* drift7, double* kick8);

/* Diagnostics of Sect. 5.1 per cluster, written to the DEVICE array out[B][20] (float64):
 *   0 K = 1/2 sum m |v|^2     1 W = 1/2 sum m_i pot_i     2 Uext = sum m Phi_ext (field clusters)
 *   3 E = K + W + Uext         4..6 P = sum m v             7..9 L = sum m x cross v
 *   10..12 torque = sum m x cross a_ext(x) (Eq. 8)          13 M = sum m
 *   14..16 F = sum m a_int     17 |F|                       18 sum m |a_int|
 *   19 1.0 if any of entries 0..18 is not finite, else 0.0
 * a_int is the internal (pair) acceleration of Eq. 5 without the galaxy field; the pair forces of
 * Eq. 2 are antisymmetric, so F is zero up to the rounding of the pair arithmetic, and |F| over
 * sum m |a_int| measures it.  The pair potential and a_int are evaluated in the system's precision
 * mode (use NB_FP64 for energy-error measurements).  Reductions run in FP64 in a fixed order
 * (bitwise reproducible).  Asynchronous: the non-finite flag stands in for NB_ERR_NONFINITE, which
 * the call cannot return because it does not wait for its kernels. */
int nbody_energy(nbody_ctx* ctx, const nbody_system* sys, const double* pos, const double* vel,
                 const double* mass, double* out, void* ws, size_t ws_bytes, void* stream);

/* Message for the last failing call on this thread ("" if none). */
const char* nbody_last_error(void);

/* ---- Tuning and instrumentation (not part of the method) ---------------------------------- */

/* Pair-kernel launch shape for one precision family and cluster-size class:
 *   prec  NB_FP32 / NB_FP32C (share a kernel), NB_FP32DS, NB_FP64 or NB_FP32DL
 *   nclass 0: largest cluster < 2048 particles, 1: < 32768, 2: < 131072, 3: larger
 *   k     i-particles per lane; waves_per_group  wavefronts sharing the same i-particles, each
 *         taking 1/waves_per_group of every j-tile; (k, waves_per_group) in {(1,1), (1,2), (1,4),
 *         (2,2), (2,4)}; one work item covers 256 k / waves_per_group particles
 *         (NB_FP32DL: all but (1,1))
 *   tile  j-records per LDS tile (128 or 256); FP32 partial sums are folded into FP64 after every
 *         tile/waves_per_group terms, so tile and waves_per_group change the last bits of FP32-mode
 *         results while k and blocks_per_cu never do (in NB_FP32DL k does too: it sets the work
 *         item whose bounding box the local coordinates are centred on)
 *   blocks_per_cu  persistent blocks per compute unit (1..8)
 *   phased  FP32 families only: full tiles are evaluated in groups of 8 pair terms whose
 *         reciprocal square roots issue back to back (shapes (1,4,256), (2,2,256), (2,4,*));
 *         the arithmetic of every term is unchanged
 * Returns NB_ERR_ARG for combinations that are not compiled in. */
typedef struct {
  int32_t k, waves_per_group, tile, blocks_per_cu, phased;
} nbody_tile;
int nbody_set_tile(nbody_ctx* ctx, int32_t prec, int32_t nclass, nbody_tile tile);
int nbody_get_tile(const nbody_ctx* ctx, int32_t prec, int32_t nclass, nbody_tile* tile);

/* Step graphs (enable = 1, the default; 0 launches every kernel directly).  Replaying a captured
 * step halves the gap between consecutive kernels on gfx950 under ROCm 7 (3.7 against 7.4 us in a
 * kernel trace of the N = 1024 leapfrog), which is what bounds small systems.  When on, nbody_step_leapfrog /
 * nbody_step_sym6 calls with nsteps >= 2 capture the kernels of up to 8 steps into a HIP graph, and
 * nbody_substeps calls with nrounds >= 2 capture their rounds, once per argument set (a change of
 * any pointer, dt, system layout or launch shape recaptures; 8 graphs are cached), and replay them
 * on the caller's stream.  Results are bitwise those of the direct launches.  Disabled automatically while per-kernel timing is on. */
int nbody_use_graphs(nbody_ctx* ctx, int enable);

/* Per-kernel timing with HIP events recorded on the call's stream around every pair-kernel
 * launch (enable = 1) or off (0, the default).  nbody_timing_read returns the summed duration
 * in milliseconds and the number of timed launches since the last read, waiting for the
 * recorded events to complete; it resets the counters. */
int nbody_timing_enable(nbody_ctx* ctx, int enable);
int nbody_timing_read(nbody_ctx* ctx, double* ms_total, int64_t* launches);

/* Pair interactions one force evaluation of `sys` performs: sum_b N_b^2 (j = i counted). */
int64_t nbody_interactions(const nbody_system* sys);

#ifdef __cplusplus
}
#endif
#endif /* NBODY_H */
