// Internal structures shared by the kernels and the host runtime.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace qg {

// Phase operations.  A right-hand-side evaluation, the B sub-step, the
// entry/exit transforms, the mask precompute, the diagnostics and the
// adjoint are all sequences of three kernel kinds: a column-inverse pass
// (spectral fields -> mixed (y, kx) layout), a row pass (c2r, pointwise
// physics, r2c) and a column-forward pass (mixed -> spectral, combine).
enum Op : int {
  OP_RHS = 0,       // A sub-step right-hand side (per closure)
  OP_B = 1,         // penalization + sponge sub-step
  OP_ENTRY = 2,     // physical omega -> projected spectral state
  OP_EXIT = 3,      // spectral state -> physical omega
  OP_MASKFWD = 4,   // chi -> half spectrum (full set minus Nyquist lines)
  OP_MASKGRAD = 5,  // spectral gradient of chi -> S E, S E_x, S E_y tables
  OP_DIAG = 6,      // diagnostics at the state
  OP_ADJ_RHS = 7,   // adjoint of the right-hand side (static closures)
  OP_ADJ_B = 8,     // adjoint of the B sub-step
  OP_ADJ_EXIT = 9,  // adjoint of the exit transform (physical -> spectral)
  OP_ADJ_ENTRY = 10,// adjoint of the entry transform (spectral -> physical)
  OP_PEN = 11,      // AB2CN: D curl(chi u) of the total velocity
  OP_SPONGE = 12,   // AB2CN: omega* - dt sigma chi_s (3/2 omega* - 1/2 omega**)
  OP_GTERMS = 13,   // SGS analysis: D FFT(J) + (1/eta) D curl(chi u) + sigma D FFT(chi_s omega)
  OP_CLIPF = 14     // pointwise clip of the dynamic coefficient: sums of max(H, 0) M and M^2 on the grid
};

// RK stage code of the AB2CN update in the column-forward / combine passes
constexpr int AB2CN_STAGE = 9;
// coefficient slot of the AB2CN history flag (0: no history yet)
constexpr int AB2CN_FLAG_SLOT = 30;
// stage code of the right-hand-side pass that writes the closure's term
// C D div(base grad omega) instead of updating the state
constexpr int SGS_STAGE = 10;
// coefficient slot holding C of the stage whose adjoint is being formed
// (dynamic closures)
constexpr int ADJ_C_SLOT = 31;

// Per-member constants, resident on the device.
struct MemberDev {
  char* base;            // start of the member's workspace region
  long long omega_off;   // byte offset of the member in flat user fields
  int user_index;        // position of the member in the caller's order
  double two_pi_lx, two_pi_ly;
  double dt, beta, inv_re, mu, u_in, v_in;
  double dt2, dt3, dt6;   // dt/2, dt/3, dt/6 of the RK4 weights, formed on the host
  double coef_static;    // (c Delta)^2 or (c Delta)^3; 0 without closure
  double dcoef_dc;       // d coef / d c
  double r_test;         // (Delta~/Delta)^p for the dynamic closures
  double lowk2;          // |k|^2 bound of the double-precision Poisson inversion
  double pen_a;          // dt / eta (0 without obstacle)
  double pen_c;          // AB2CN: the constant split off chi in the penalty's curl (the mask's mean)
  double sponge_a;       // dt * sigma
  double inv_n;          // 1 / (nx ny)
  double inv_delta;      // 1 / Delta = nx / lx
  long long test_lim;    // min(Mx ny, My nx)^2 of the integer test-filter test
  int test_r2;           // test_ratio^2
  int test_kx;           // columns m_x < test_kx hold the test-filtered modes
  int closure;
  int clip_mode;         // 0: C = max(<HM>, 0)/<M^2>; 1: C = <max(H, 0) M>/<M^2>
  // byte offset from base to the tables S E, S E_x, S E_y the B sub-step
  // reads: the member's own, or those of an earlier member of its group
  // with the same masks and the same dt/eta and dt sigma (equal bits)
  long long tab_off;
};

// Byte offsets of the buffers inside every member region of a group
// (members of a group share sizes, hence offsets).
struct RegionLayout {
  long long wn, acc, x, jsp, qsp, chih, mf, mp, phys, part, coef, dpart;
  long long ab_pen, ab_hist, ab_wss;               // AB2CN: D curl(chi u), explicit terms, omega**
  long long adj_lam, adj_lacc, adj_lk, adj_store;  // adjoint buffers
  long long clip_h, clip_m;                         // pointwise clip: the H and M spectra of the stage
  long long adj_hmq, adj_cs;                        // dynamic-closure adjoint: H, M, Q and (C, <HM>, <M^2>) per stage
  long long adj_a, adj_b, adj_e;                    // ... the cotangents of H and M, the coefficient's term
  long long total;
};

// Arguments of one launch (one phase of one size group).
struct Phase {
  const MemberDev* mem;
  int m0;                 // first member of the group in the member table
  int nx, ny, lognx, logny;
  int kxn, myh, kyn, kxp; // retained kx count, |m_y| bound, compact y count, row pitch
  int W, logW;            // strip width of the column-forward pass (and MP layout)
  int Wi, logWi;          // strip width of the column-inverse pass
  int mfp;                // row pitch of the row-major MF layout
  int RP, logRP;          // row pairs per row block
  int nf;                 // number of fields of a column-inverse launch
  int stage;              // RK stage 1..4 (0: not a stage)
  int nparts;             // partial-sum slots written by the column-forward pass
  long long o_in, o_in2, o_out, o_aux;  // op-specific byte offsets
  long long o_ab_pen, o_ab_hist;        // AB2CN: penalization curl, explicit-term history
  long long o_mf, o_mp, o_phys, o_part, o_coef, o_dpart;
  const void* twx;        // twiddles exp(-2 pi i m / nx)
  const void* twy;        // twiddles exp(-2 pi i m / ny)
  void* user;             // user physical output (exit, diag nu_e)
  const void* user_in;    // user physical input (entry)
  long long user_stride;  // elements between saves (unused: 0)
  // dynamic-closure adjoint (all 0 elsewhere).  adj_dyn: the forward
  // column pass of a dynamic closure keeps H (o_h) and M (o_m) and the
  // combine keeps (C, <HM>, <M^2>) at o_cs; in the adjoint right-hand-side
  // pass, C (ADJ_C_SLOT) and the cotangents -T a, -T b of H and M (o_a,
  // o_b) are folded into the pass's input and the term at o_e is added.
  // adj_mode 1: the transport pass at the test-filtered stage input with
  // the cotangents a, r b, its result test-filtered to o_e.
  int adj_dyn, adj_mode;
  long long o_h, o_m, o_a, o_b, o_e, o_cs;
  // profiling runs only: HIP events bound to this launch's dispatch (begin,
  // end); null otherwise
  void* ev0;
  void* ev1;
  // tuning choices of the compile-time engines of the step's passes: pass
  // schedule of the row transforms (rsch) and of the column transforms
  // (csch), with the twiddle tables of schedule 1 (twx1, twy1); row pairs
  // per block of the row pass (rpb); wave-synchronous row transforms (rwv:
  // one wave per transform); wave-synchronous radix-16 transforms of the
  // FP32 1024-point forward columns of the dynamic closures (cwv)
  int rsch, csch, rpb, rwv, cwv;
  const void* twx1;
  const void* twy1;
  const void* twx2;       // the row and column tables of schedule 2 (radix 16)
  const void* twy2;
  // dynamic LDS bytes of the launch (set by the launcher; read by the LDS
  // poison of debug builds)
  unsigned lds_bytes;
  // stamp builds only (QG_STAMPS; null elsewhere): the per-wave phase
  // stamps of qg_stamp_steps
  unsigned long long* stamps;
};

// Stamp builds: QG_STAMP_KINDS kernels (0 the right-hand side's row pass,
// 1 its column-inverse pass, 2 its column-forward pass and 3 the combine
// of the dynamic closures), QG_STAMP_WAVES waves each (member 0), 8 slots
// per wave: real-time counter values at the kernel's phase boundaries,
// slot 7 the wave's hardware ids (HW_ID in the low, XCC_ID in the high
// 32 bits).
constexpr int QG_STAMP_KINDS = 4;
constexpr int QG_STAMP_WAVES = 8192;
constexpr size_t QG_STAMP_BYTES = (size_t)QG_STAMP_KINDS * QG_STAMP_WAVES * 8 * sizeof(unsigned long long);

// Column passes: a strip tile of W * ny elements (4096 float2 or 2048
// double2, 32 KiB, unless one column is longer) with 8 elements per thread,
// i.e. W * ny / 8 threads (at most 512).
constexpr int COL_EPT = 8;
constexpr int COL_MAX_THREADS = 512;
__host__ __device__ constexpr int col_tile_elems(bool dbl) { return dbl ? 2048 : 4096; }
constexpr int COMBINE_THREADS = 512;

// Launchers (defined in qg_kernels.hip).  Each returns hipGetLastError().
hipError_t launch_colinv(bool dbl, int op, int closure, const Phase& P, int nmem, hipStream_t s);
hipError_t launch_row(bool dbl, int op, int closure, const Phase& P, int nmem, hipStream_t s);
hipError_t launch_colfwd(bool dbl, int op, int closure, const Phase& P, int nmem, hipStream_t s);
hipError_t launch_combine(bool dbl, int op, const Phase& P, int nmem, hipStream_t s);
hipError_t launch_diag_spectral(bool dbl, const Phase& P, int nmem, hipStream_t s);
hipError_t launch_diag_final(const Phase& P, int nmem, int nrowblocks, int nspecblocks,
                             double* out, int out_member0, hipStream_t s);
hipError_t launch_dyn_coef(const Phase& P, int nmem, int slot, hipStream_t s);
hipError_t launch_adj_grad_c(const Phase& P, int nmem, int nrowblocks, double* grad_c,
                             int mode, hipStream_t s);
int row_launch_blocks(bool dbl, int op, int closure, const Phase& P);
// whether the field-parallel row kernel (the one that takes two levels in
// one launch) runs op for these sizes
bool row_two_levels_ok(bool dbl, int op, int closure, const Phase& P);
hipError_t launch_spec_axpy(bool dbl, const Phase& P, int nmem, long long o_dst,
                            long long o_src, double a, int zero_first, hipStream_t s);
hipError_t launch_spec_copy(bool dbl, const Phase& P, int nmem, long long o_dst,
                            long long o_src, hipStream_t s);
hipError_t launch_ab2cn_finish(bool dbl, const Phase& P, int nmem, hipStream_t s);
// dynamic-closure adjoint: s = <lambda, Q> (lambda at o_in2, Q at o_aux),
// then with the kept C, <HM>, <M^2> (o_cs) the cotangents
// a = (s/<M^2>) M, b = (s/<M^2>)(H - 2 C M) of H and M (o_h, o_m)
hipError_t launch_adj_dyn_prep(bool dbl, const Phase& P, int nmem, hipStream_t s);

// One member pair of the LES filter: FR D-compact spectrum -> coarse
// full-set compact spectrum.
struct FilterArgs {
  const void* src;             // FR state of the member
  void* dst;                   // coarse full-set spectrum of the member
  int kxn_f, kyn_f, myh_f;     // FR 2/3 set
  int kxn_c, kyn_c, myh_c;     // coarse full set (Nyquist lines excluded)
  double two_pi_lx, two_pi_ly;
  double width2;               // (delta Delta_FR)^2
  double kc2;                  // (pi / Delta_FF)^2
  double inv_d2;               // 1 / delta^2
};
hipError_t launch_filter_les(bool dbl, const FilterArgs& A, hipStream_t s);
// nblk blocks per member; the member's dpart area must hold 5 nblk doubles
hipError_t launch_pcc(bool dbl, const Phase& P, int nmem, int nblk, const void* a, const void* b, double* out,
                      hipStream_t s);
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s);
// one member's constants into the device table at dst
hipError_t launch_put_member(MemberDev* dst, const MemberDev& m, hipStream_t s);
// the per-pass twiddle table of length-2^logn transforms, schedule sch
hipError_t launch_twiddle_table(bool dbl, void* dst, int logn, int sch, hipStream_t s);
// whether the SGS-analysis pass (field-parallel row and column kernels at
// strip width 1) fits the group's sizes
bool gterms_ok(bool dbl, const Phase& P);

// Field counts per phase and closure.
__host__ __device__ constexpr int rhs_fields(int cl) { return cl == 0 || cl == 2 ? 4 : cl == 1 ? 6 : cl == 4 ? 8 : 12; }
__host__ __device__ inline int rhs_products(int cl) { return cl == 0 ? 1 : (cl == 1 || cl == 2) ? 3 : 6; }
__host__ __device__ inline bool smag_family(int cl) { return cl == 1 || cl == 3; }
__host__ __device__ constexpr bool dynamic_closure(int cl) { return cl == 3 || cl == 4; }

// Fields (thread groups) and products of the field-parallel row pass.
__host__ __device__ constexpr int rowp_nb(int op, int cl) {
  return (op == OP_B || op == OP_ADJ_B) ? 3
       : op == OP_GTERMS ? 5
       : op == OP_CLIPF ? 2
       : (op == OP_PEN || op == OP_SPONGE) ? 2
       : op == OP_ADJ_RHS ? ((cl == 1 || cl == 3) ? 6 : 4) + (cl == 0 ? 1 : 3)
       : ((cl == 1 || cl == 3) ? 6 : 4);
}
__host__ __device__ constexpr int rowp_np(int op, int cl) {
  return op == OP_ADJ_RHS ? ((cl == 1 || cl == 3) ? 6 : 4)
       : op == OP_ADJ_B ? 3
       : op == OP_GTERMS ? 4
       : op == OP_CLIPF ? 0
       : op == OP_PEN ? 2
       : (op == OP_B || op == OP_SPONGE || cl == 0) ? 1 : 3;
}

}  // namespace qg
