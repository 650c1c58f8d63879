/*
 * qg.h -- C ABI of the MI355X (gfx950) pseudo-spectral QG time step.
 *
 * One step advances the non-dimensional beta-plane quasi-geostrophic
 * vorticity equation (Sec. II-A, Eq. 1)
 *     d omega/dt + J(psi, omega) = (1/Re) lap omega - mu omega - beta psi_x
 *                                  + Pi + F_obs + F_sponge,   omega = lap psi,
 * on a doubly periodic nx-by-ny grid with a Fourier pseudo-spectral method
 * and 2/3 de-aliasing (Sec. II-C).  Pi = div(nu_e grad omega) is the
 * eddy-viscosity closure (Eq. 8): Smagorinsky (Eq. 9), Leith (Eq. 12) or
 * their dynamic variants with the Germano identity and Lilly's least
 * squares (Eqs. 10-11, 13).  F_obs is Brinkman volume penalization with
 * porosity eta and mask chi_obs (Sec. II-B, Eq. 2); F_sponge relaxes omega
 * with rate sigma = 1/eta_sponge on the ramp chi_sponge (Sec. II-D, Eq. 3);
 * a uniform inflow (u_in, v_in) is added to the zeroth Fourier mode of the
 * velocity (Sec. II-D).
 *
 * Time step (splitting of Sec. II-E), selected per member by `scheme`:
 *  QG_SCHEME_RK4: classical RK4 over advection, beta, viscosity and
 *    closure, then an exactly integrated sub-step applying the penalization
 *    (curl of u <- exp(-dt chi/eta) u, product rule) and then the sponge
 *    (omega <- exp(-dt sigma chi_s) omega), evaluated pointwise in physical
 *    space and projected back onto the 2/3 set;
 *  QG_SCHEME_AB2CN: the paper's own scheme (Eq. 4): Crank-Nicolson on the
 *    linear terms (viscosity, friction, beta), second-order Adams-Bashforth
 *    on the Jacobian, the closure and the penalization curl(chi u / eta),
 *    then the sponge by Adams-Bashforth 2 on omega* and the previous step's
 *    omega**.  Explicit penalization needs eta > dt (checked).  The scheme carries
 *    history inside the handle (the previous explicit terms and omega**):
 *    the first step after qg_init is forward Euler on the explicit parts,
 *    and later qg_step calls continue the sequence, so the omega passed in
 *    must be the one the previous call returned.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Fields are row-major (ny, nx), x contiguous, element type float when
 *    precision == 32 and double when precision == 64.  Members of a batch
 *    are concatenated in the order given to qg_init.
 *  - All device pointers are owned by the caller.  The library keeps the
 *    workspace pointer from qg_init until qg_destroy and never frees it; it
 *    keeps no other caller pointer beyond the call.
 *  - Calls enqueue work on the given HIP stream (hipStream_t passed as
 *    void*, NULL = default stream) and return without synchronising, except
 *    qg_init and qg_autotune, which synchronise their stream.
 *  - Return codes are QG_* below; no C++ exception crosses this boundary.
 *    On failure qg_last_error() returns a message (thread-local).
 *  - One host thread at a time per handle.
 */
#ifndef QG_H
#define QG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    QG_OK = 0,
    QG_EINVAL = 1,        /* bad argument or parameter value                  */
    QG_EUNSUPPORTED = 2,  /* valid but not implemented (sizes, clip_mode...)  */
    QG_EWORKSPACE = 3,    /* workspace missing, misaligned or too small       */
    QG_EHIP = 4,          /* a HIP runtime call failed (message has details)  */
    QG_ESTATE = 5         /* call not valid in the handle's current state     */
};

enum {
    QG_SCHEME_RK4 = 0,     /* RK4 + exactly integrated penalization/sponge    */
    QG_SCHEME_AB2CN = 1    /* AB2CN + AB2 sponge, Sec. II-E, Eq. 4            */
};

enum {
    QG_CLOSURE_NONE = 0,
    QG_CLOSURE_SMAG = 1,   /* nu_e = (c Delta)^2 |S|,  Eq. 9                   */
    QG_CLOSURE_LEITH = 2,  /* nu_e = (c Delta)^3 |grad omega|, Eq. 12          */
    QG_CLOSURE_DSMAG = 3,  /* dynamic Smagorinsky, Eqs. 10-11                  */
    QG_CLOSURE_DLEITH = 4  /* dynamic Leith, Eq. 13                            */
};

/* Parameters of one member (Sec. II-A..E, III-A).
 *  nx, ny       grid, powers of two in [32, 4096]; dx = lx/nx must equal
 *               dy = ly/ny to 1e-12 relative (Delta = dx, Eq. 9)
 *  lx, ly       domain size
 *  beta, re, mu beta-plane gradient, Reynolds number (re <= 0 or inf means
 *               no molecular viscosity), bottom friction (Eq. 1)
 *  u_in, v_in   uniform inflow added to the zeroth velocity mode
 *  eta          Brinkman porosity (Eq. 2), must be > 0; inf disables the
 *               obstacle.  QG_SCHEME_AB2CN members need eta > dt (the
 *               explicit penalization's stability bound, Sec. II-E);
 *               qg_init and qg_workspace_bytes return QG_EINVAL otherwise
 *  sponge_sigma 1/eta_sponge (Eq. 3); 0 disables the sponge
 *  dt           time step
 *  c            static c_S or c_L (ignored by the dynamic closures)
 *  closure      QG_CLOSURE_*
 *  precision    32 or 64: arithmetic and storage type of the step
 *  test_ratio   Delta~/Delta of the test filter, integer in {2, 3, 4};
 *               the test filter keeps |k| <= k_max / test_ratio with k_max
 *               the largest retained wavenumber (Sec. III-A, dynamic models)
 *  clip_mode    dynamic closures only (Sec. III-A, the clip of H).
 *               0: C = max(<HM>, 0)/<M^2>, the clip applied to the
 *               average.  1: C = <max(H, 0) M>/<M^2>, H clipped at every
 *               grid point (C may then be negative: the ratio is not
 *               clipped again); needs nx >= 64 (and nx <= 2048 in 64-bit
 *               runs) and has no adjoint (qg_adjoint_step returns
 *               QG_EUNSUPPORTED for a handle that holds it).
 *  fp64_lowk    in 32-bit runs, modes with |k| <= fp64_lowk invert the
 *               Poisson equation in double precision
 *  scheme       QG_SCHEME_*.  QG_SCHEME_AB2CN needs nx >= 64 (and
 *               nx, ny <= 2048 in 64-bit runs); it has no adjoint.        */
typedef struct {
    int32_t nx, ny;
    double lx, ly, beta, re, mu, u_in, v_in, eta, sponge_sigma, dt, c;
    int32_t closure;
    int32_t precision;
    double test_ratio;
    int32_t clip_mode;
    int32_t fp64_lowk;
    int32_t scheme;
} qg_params;

typedef struct qg_handle qg_handle;

/* Bytes of device workspace needed for n_members members (params[i] each)
 * and adjoint segments of up to adj_segment_k steps (0: no adjoint).
 * Writes *bytes.  Validates the parameters as qg_init does. */
int qg_workspace_bytes(const qg_params* params, int32_t n_members,
                       int32_t adj_segment_k, size_t* bytes);

/* Build a handle for n_members members.
 *  chi_obs[i], chi_sponge[i]: device pointers to member i's masks (Eq. 2 and
 *      Eq. 3), (ny, nx) of the member's precision; copied into the workspace.
 *  workspace, ws_bytes: caller-owned device buffer, 256-byte aligned, at
 *      least qg_workspace_bytes(...) bytes (same adj_segment_k).
 * Precomputes the penalization tables E = exp(-dt chi/eta), E_x, E_y (from
 * the spectral gradient of chi) and S = exp(-dt sigma chi_sponge) on the
 * GPU.  Synchronises hip_stream.  Members may differ in every parameter;
 * members of equal (nx, ny, precision, closure) are launched together.
 * Members of such a group given the same chi_obs and chi_sponge pointers
 * and equal dt/eta and dt sigma have equal tables: the step reads the
 * first such member's copy for all of them. */
int qg_init(const qg_params* params, int32_t n_members,
            const void* const* chi_obs, const void* const* chi_sponge,
            void* workspace, size_t ws_bytes, int32_t adj_segment_k,
            void* hip_stream, qg_handle** out);

/* Advance every member nsteps steps in place.  omega: flat device buffer of
 * all members.  On entry omega is projected onto the 2/3 set with its mean
 * removed; the state stays spectral inside the call.  If save_every > 0,
 * omega is written to ckpt_out (n_saves x all members, flat) after every
 * save_every steps, and the run continues from that written field, so a run
 * restarted from a checkpoint repeats the original bit for bit.
 * use_graph != 0 replays a captured hipGraph of the step sequence (captured
 * on library-owned streams, one branch per size group so that the groups
 * run concurrently -- a handle of a single size group of two or more
 * members as two branches of half the members each; ordered after, and
 * before, the caller's stream work by events).  Graph and eager steps give
 * the same bits. */
int qg_step(qg_handle* h, void* omega, int64_t nsteps, int32_t save_every,
            void* ckpt_out, int32_t use_graph, void* hip_stream);

/* Discrete adjoint of qg_step over one segment (QG_SCHEME_RK4 only).
 * omega_ckpt: omega at the segment start (as saved by qg_step);
 * lambda: on entry dL/d omega at the segment end, on return dL/d omega at
 * the segment start (both physical, same layout as omega);
 * grad_c_dev: n_members doubles on the device; dL/dc of each member is
 * ADDED to it (0 for the dynamic closures, which have no c).
 * nsteps <= adj_segment_k given to qg_init.
 * For the dynamic closures the coefficient C = max(<HM>, 0)/<M^2> of every
 * stage is differentiated with respect to the stage input (through H and
 * M, Eqs. 10-11, 13); where the clip sets C = 0 its derivative is 0. */
int qg_adjoint_step(qg_handle* h, const void* omega_ckpt, void* lambda,
                    int64_t nsteps, double* grad_c_dev, void* hip_stream);

/* The LES filter of Sec. III, H_full = interpolation onto the LES grid o
 * cut-off at |k| > pi/Delta_FF o Gaussian exp(-k^2 (delta Delta_FR)^2 / 6),
 * for every member pair: member i of `fr` holds the fully-resolved grid,
 * member i of `les` the same domain coarsened by delta (a power of two
 * >= 2, equal in x and y, same precision).  omega_fr: flat FR fields (fr's
 * layout), projected onto the FR 2/3 set on entry; omega_ff: the filtered
 * fields on the LES grids (les's layout; the coarse Nyquist modes are
 * zero).  Uses both workspaces as scratch: call between qg_step calls, not
 * during one (the handles' states live in the caller's omega). */
int qg_filter_les(qg_handle* fr, qg_handle* les, const void* omega_fr, void* omega_ff,
                  void* hip_stream);

/* The ideal subgrid-scale forcing of the filtered QG equations (Sec. III)
 * and the closure's model of it (Sec. IV, the a-priori term), for every
 * member pair of `fr` and `les` (the pairing rules of qg_filter_les):
 *   G(omega) = D FFT(J) + (1/eta) D curl(chi u) + sigma D FFT(chi_s omega),
 *   pi_ff    = P_D [ G_les(omega_bar) - H_full(G_fr(omega)) ],
 * with J the advection by the total velocity, u the total velocity, D the
 * 2/3 set of each grid, P_D the projection onto the LES one, and
 * omega_bar = P_D H_full(omega): the forcing that makes an LES tendency on
 * its 2/3 set equal the filtered FR tendency.  G_fr takes eta, sigma,
 * chi, chi_s and the inflow of the fr member, G_les those of the les
 * member (give it H_full of the FR masks for the paper's definition).
 * pi_model (may be NULL): C D div(base grad omega_bar), the les member's
 * closure at omega_bar (C from omega_bar for the dynamic closures, zero
 * without closure).  omega_bar (may be NULL): omega_bar itself.
 * omega_fr: flat FR fields in fr's layout; outputs: flat fields in les's
 * layout.  Sizes: 64 <= nx <= 1024 on both grids, ny <= 1024 in 64-bit and
 * ny <= 2048 in 32-bit runs; else QG_EUNSUPPORTED.  Uses both workspaces
 * as scratch, like qg_filter_les. */
int qg_ideal_sgs(qg_handle* fr, qg_handle* les, const void* omega_fr, void* pi_ff,
                 void* pi_model, void* omega_bar, void* hip_stream);

/* The closure's term Pi = C D div(base grad omega) of every member at the
 * physical fields omega (projected onto the 2/3 set on entry; C from omega
 * for the dynamic closures, zero without closure): the a-posteriori model
 * term Pi_LES of Sec. IV when omega is an LES state.  omega, out: flat
 * device fields in the handle's layout.  Uses the workspace as scratch,
 * like qg_filter_les. */
int qg_closure_term(qg_handle* h, const void* omega, void* out, void* hip_stream);

/* Pattern (Pearson) correlation of two fields per member (Sec. IV):
 * out_dev[i] = <(a - <a>)(b - <b>)> / sqrt(<(a - <a>)^2> <(b - <b>)^2>) over
 * member i's grid, <.> the grid mean, in double precision.  a, b: flat
 * device fields in the handle's layout; out_dev: n_members doubles. */
int qg_pcc(qg_handle* h, const void* a, const void* b, double* out_dev, void* hip_stream);

/* Replace the closure coefficient c of every member (c_host: n_members
 * doubles on the host; ignored for members without a static closure).  The
 * update is ordered on hip_stream after previously enqueued work; replays
 * of captured graphs see the new values. */
int qg_set_coef(qg_handle* h, const double* c_host, void* hip_stream);

/* Diagnostics at omega: for each member 8 doubles
 *   [energy 1/2<|grad psi|^2>, enstrophy 1/2<omega^2>, C, nu_min, nu_mean,
 *    nu_max, CFL = max(|u|+|v|) dt/Delta, nonfinite flag]
 * into out_dev (device, n_members x 8).  nu_e_out (nullable): the eddy
 * viscosity field nu_e = C base, flat like omega. */
int qg_diag(qg_handle* h, const void* omega, double* out_dev, void* nu_e_out,
            void* hip_stream);

/* Choose the launch configuration of every size group by timing: the
 * tunables are the strip width of the column-forward pass (W) and of the
 * column-inverse pass (Wi), the radix schedule of the compile-time row and
 * column transforms (rows and columns of 256, 512 or 1024 points; schedule
 * 0: radix 8 then 4 or 2, e.g. 1024 = 8 8 8 2; schedule 1: radix 4s
 * between radix-8 first and last passes, e.g. 1024 = 8 4 4 8; schedule 2,
 * 1024-point rows with one wave per transform only: 8 16 8), the row pairs
 * per block of the step's row pass (1 or 2) and its synchronisation
 * (block-wide passes of 8 points per thread, or one wave per transform, 16
 * points per thread at 1024, with block barriers only around the pointwise
 * products; the same choice gives the FP32 1024-point columns of the
 * dynamic closures' forward pass one wave per transform under the radix-16
 * schedule).  All combinations of the admissible values are searched
 * jointly: each is captured as a graph of four steps of the group and timed
 * round-robin three times (after two warm-up rounds) on a stream of the
 * tuner's own, and the fastest is kept.  The choice is cached in the flat
 * JSON file at cache_path (nullable: no file) under the group's key with
 * the suffixes /fwd, /inv, /rsched, /csched, /rpb, /rwave; a tunable found in the
 * cache is taken as given and only the others are searched.  Every choice
 * computes the same step (to rounding).  The timed steps run on the
 * workspace: the spectral state is not meaningful afterwards (the next
 * qg_step enters omega again) and the history of QG_SCHEME_AB2CN members
 * starts again (forward-Euler first step).  Synchronises hip_stream. */
int qg_autotune(qg_handle* h, const char* cache_path, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): qg_step
 * of one member without a handle or a caller workspace.  p, chi_obs,
 * chi_sponge and omega are as for qg_init / qg_step (one member; device
 * pointers of the member's precision); omega is advanced nsteps RK4 steps
 * in place, with the launches of qg_step's eager path and the library's
 * default launch configuration (no tuning, no graph).  The workspace is a
 * static device array of 64 MiB inside the library, one per GPU, held until
 * the process ends: every call sets it up afresh on hip_stream (member
 * constants, twiddle tables computed on the device, mask tables) and no
 * call allocates, frees or synchronises.  Every call on a GPU shares that
 * GPU's array, so calls that overlap on one GPU (concurrent streams or
 * threads) race and must be serialised by the caller.
 * Returns QG_EUNSUPPORTED when the member's workspace exceeds the array
 * (64 MiB holds every closure up to 512 x 512 in FP64 and 1024 x 512 in
 * FP32) or its scheme is not QG_SCHEME_RK4; the other errors as qg_init. */
int qg_step_noalloc(const qg_params* p, const void* chi_obs, const void* chi_sponge, void* omega,
                    int64_t nsteps, void* hip_stream);

/* The launch configuration of every member's size group: out (host,
 * n_members x 6 int32) receives W, Wi, row schedule, column schedule, row
 * pairs per block and wave-synchronous row transforms (see qg_autotune). */
int qg_tuning(const qg_handle* h, int32_t* out);

/* Profiling: qg_step(h, omega, nsteps) without graphs (the same launches in
 * the same order on hip_stream, omega updated in place), where every launch
 * of one kind of step kernel is bound to a pair of HIP events that carry
 * its dispatch's own begin and end times.  kind: 0 column-inverse pass of
 * the right-hand side, 1 its row pass, 2 its column-forward pass, 3 the
 * dynamic combine (dynamic closures only), 4 column-inverse pass of the B
 * sub-step, 5 its row pass, 6 its column-forward pass; every size group's
 * launches of that kind are timed.  ms (host, max_launches floats) receives the duration of
 * each of the first max_launches such launches in milliseconds and
 * *n_launches their number.  RK4 members only (QG_EUNSUPPORTED otherwise).
 * Synchronises hip_stream; the library creates and destroys the events. */
int qg_profile_steps(qg_handle* h, void* omega, int64_t nsteps, int32_t kind, float* ms,
                     int32_t max_launches, int32_t* n_launches, void* hip_stream);

/* Phase stamps, for the debug build libqg_stamps.so (compiled with
 * QG_STAMPS; every other build returns QG_EUNSUPPORTED): qg_step(h, omega,
 * nsteps) without graphs, as qg_profile_steps, during which lane 0 of every
 * wave of member 0 of the four right-hand-side kernels (kind 0 the row
 * pass, 1 the column-inverse pass, 2 the column-forward pass and 3 the
 * combine of the dynamic closures) writes the GPU's 100 MHz real-time
 * counter at the kernel's phase boundaries into stamps (device memory of
 * at least 4 x 8192 x 8 uint64, 2 MiB, to be zeroed by the caller): wave w
 * (the block's linear index times its waves, plus the wave in the block;
 * the first 8192 waves) of kind k at uint64 (k 8192 + w) 8 + slot.  Slots:
 * row pass 0 start, 1 loads in, 2 c2r done, 3 products formed, 4 r2c
 * done, 5 stores complete; column-inverse 0 start, 1 fields formed, 2
 * transform done, 3 stores complete; column-forward 0 start, 1 loads in, 2
 * transform done, 3 mode stores complete, 4 partial sums stored; combine 0
 * start, 1 loads in, 2 coefficient formed, 3 stores complete; slot 7 the
 * wave's hardware ids (HW_ID low, XCC_ID high 32 bits).  The passes are
 * stamped on their compile-time-length paths, the column-forward pass on
 * its one-column path (strip width 1).  A later launch of a kind
 * overwrites an earlier one's stamps (the last stage's remain).
 * RK4 members only.  Synchronises hip_stream. */
int qg_stamp_steps(qg_handle* h, void* omega, int64_t nsteps, void* stamps, size_t stamp_bytes,
                   void* hip_stream);

/* Number of members, total grid points, and the tiling chosen per member:
 * strip width of the column-forward and of the column-inverse passes
 * (each output array nullable, n_members entries). */
int qg_info(const qg_handle* h, int32_t* n_members, int64_t* total_points,
            int32_t* fwd_width_out, int32_t* inv_width_out);

void qg_destroy(qg_handle* h);
const char* qg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* QG_H */
