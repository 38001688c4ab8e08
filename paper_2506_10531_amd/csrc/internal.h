// Internal declarations shared by the host runtime (capi.hip, queue.hip) and
// the gfx950 kernels (kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace dq {

// Per (state, layer) coefficients, prepared on the device from (gamma, beta).
// The mixer e^{+i beta X} = [[c, i s], [i s, c]] is applied per qubit pair as
//   mode 0 (|tan beta| <= 1): a_self' = a_self + i t a_partner, then * c^m,
//   mode 1 (|cot beta| <  1): a_self' = a_partner - i u a_self, then * (i s)^m,
// where m is the number of qubits mixed by one pass and t = tan beta,
// u = cot beta; both forms are symmetric in the pair, so every butterfly is
// two FMAs per amplitude component.
struct LayerCoef {
  double gp;    // gamma / (2 pi): phase in revolutions per unit of C
  double tb;    // tan(beta) in mode 0, cot(beta) in mode 1
  double cb;    // cos(beta)
  double sb;    // sin(beta)
  int mode;
  int pad;
};

// One kernel pass over every tile of every state in a launch.
// Tile geometry: the k tile qubits are the low c global bits [0, c) plus the
// run [a, a + k - c) (when c == k the tile is simply bits [0, k)).  The other
// n - k bits index the tile ("block").  Mixed qubits: local bits [mixlo, k).
// Ops, in order: mixer of layer `lead` (if lead >= 0); then for every layer
// j in [ja, jb]: phase of layer j followed by the mixer of layer j.
struct PassDesc {
  int n, k, c, a;
  int mixlo;
  int lead, ja, jb;
  int flags;
  int set;     // qubit set index (planning bookkeeping)
  // Register-tile kernel (complex64, 14-qubit tiles) only: kind 1 = tile
  // [0, 14) fully mixed, kind 2 = tile [0, 4) + [a, a + 10) mixing local
  // bits [mixlo, 14); 0 = the LDS-tile kernel.  The register-tile kernel
  // leaves each mixer's scalar factor (c^m or (i s)^m) pending and folds it
  // into the next phase; pend_* list the mixer ops (layer, qubit count)
  // whose factors are still pending when this pass starts.
  int kind;
  int pend_n;
  int pend_layer[2];
  int pend_m[2];
};

enum PassFlags {
  F_INIT = 1,      // start from |+> instead of reading the state
  F_WRITE = 2,     // write the tile back
  F_REDUCE = 4,    // per-tile partial sums of |psi|^2 C and |psi|^2
  F_PROBS = 8,     // write |psi|^2 (state precision) to `probs`
  F_LAMBDA = 16,   // gradient: fuse the adjoint sweep of this pass (last pass)
};

struct Plan {
  int sets = 0;
  int K = 0;       // tile-qubit limit used
  int c = 0;       // contiguous low qubits per tile
  int k[4] = {0, 0, 0, 0};
  int a[4] = {0, 0, 0, 0};
  int npass = 0;
  PassDesc pass[2 * 64 * 3 + 4];
};

// Builds the pass sequence.  kmax: qubits per LDS tile (13/14 for one
// complex128/complex64 tile, one less when two tiles share LDS).
bool make_plan(int n, int p, int kmax, int cpref, Plan* out);
// Plan for the register-tile kernels: every tile has K qubits; set 0 =
// [0, K), set i >= 1 = [0, C_i) + a run of K - C_i high bits of which it mixes
// its share of [K, n).  The number of sets is that for C_i = C; each set then
// takes C_i = min(cmax, K - its share).  At most 4 sets, n <= 34.
bool make_plan_regtile(int n, int p, int K, int C, Plan* out, int cmax, bool rev = false);
inline bool make_plan_regtile(int n, int p, int K, int C, Plan* out) {
  return make_plan_regtile(n, p, K, C, out, C);
}
// complex64 register-tile plan (n >= 15): K = 14, C_i from 4 to 8 (a kind-2
// set mixing tile bits [MIXLO, 14) has C_i = min(MIXLO, 8)); the first layer
// starts on the last set (rev).
bool make_plan_reg14(int n, int p, Plan* out);
// 13-qubit register-tile plan of the complex64 gradient (two sets, 14 <= n
// <= 22): set 0 = [0, 13), set 1 = [13, n) on tile bits [0, 4) + [a, a + 9).
// No pending scalars: the checkpoint passes store true-scaled states.
bool make_plan_reg13(int n, int p, Plan* out);
// The same two-set plan for any tile size K and C low bits (K = 12, C = 2:
// the complex128 gradient, 13 <= n <= 22).
bool make_plan_reg2set(int n, int p, int K, int C, Plan* out, int cmax);
inline bool make_plan_reg2set(int n, int p, int K, int C, Plan* out) {
  return make_plan_reg2set(n, p, K, C, out, C);
}

// tab: the pass's tile-independent tables, one record of TAB_BYTES per state
// (written by launch_*_tables before the passes).
hipError_t launch_fwd14_pass(const PassDesc& d, int nstates, int S, int p,
                             const void* in, void* out, uint64_t state_stride,
                             const double* W, const LayerCoef* coef,
                             double* part, void* probs, void* tab, hipStream_t stream);
constexpr size_t TAB_BYTES = 8192;

// Which layer coefficients a pass's tables use: the cot form of layer
// flip_layer flips tile bit 0 (set 0 only; -1: no flip), and the register
// factors are e^{-i 2 pi kf_sign gp K(r)} with gp of layer kf_layer (-1: none).
struct TabSpec {
  int flip_layer;
  int kf_layer;
  double kf_sign;
};

// The forward pass's spec: its lead flips bit 0, its phase layer gives KF.
inline TabSpec fwd_tab_spec(const PassDesc& d) {
  return TabSpec{d.kind == 1 && d.lead >= 0 ? d.lead : -1, d.ja <= d.jb ? d.jb : -1, 1.0};
}

// The tables of one pass, as a job of all_tables_kernel: the pass's tile
// geometry (kind; contiguous low tile bits c and run start a for kind 2) and
// its TabSpec.  kind 0: the pass needs no tables (lead-only passes).
struct TabJob {
  int8_t kind, c, a, flip, kfl, neg;
  int8_t pad[2];
};
// The most table jobs of one call.  A forward plan on m qubit sets has
// p (m - 1) + 1 passes, one job each: at most 3p + 1 = 193 at 64 layers
// (m <= 4).  A register-tile gradient runs on two sets: p + 1 passes, a
// checkpoint and an adjoint job for each but the last, 2p + 1 = 129.  The
// list travels as a kernel argument (8 bytes a job).
constexpr int MAX_TAB_JOBS = 193;
struct TabJobs {
  int njobs;
  TabJob job[MAX_TAB_JOBS];
};
inline TabJob tab_job(const PassDesc& d, const TabSpec& t, bool needed) {
  TabJob j{};
  j.kind = (int8_t)(needed ? d.kind : 0);
  j.c = (int8_t)d.c;
  j.a = (int8_t)d.a;
  j.flip = (int8_t)t.flip_layer;
  j.kfl = (int8_t)t.kf_layer;
  j.neg = (int8_t)(t.kf_sign < 0.0);
  return j;
}

// One launch computing every pass's tables of a call (all_tables_kernel), per
// geometry family; tab: J.njobs * nstates records of TAB_BYTES, pass j's at
// tab + j * nstates * TAB_BYTES.
hipError_t launch_fwd14_tables(const TabJobs& J, int n, int nstates, int S, int p,
                               const double* W, const LayerCoef* coef, void* tab,
                               hipStream_t stream);
hipError_t launch_fwd13d_tables(const TabJobs& J, int n, int nstates, int S, int p,
                                const double* W, const LayerCoef* coef, void* tab,
                                hipStream_t stream);
hipError_t launch_grad13_tables(const TabJobs& J, int n, int nstates, int S, int p,
                                const double* W, const LayerCoef* coef, void* tab,
                                hipStream_t stream);
hipError_t launch_grad12_tables(const TabJobs& J, int n, int nstates, int S, int p,
                                const double* W, const LayerCoef* coef, void* tab,
                                hipStream_t stream);
// complex128 register-tile pass on 13-qubit tiles (kind-2 sets with C = 2).
hipError_t launch_fwd13d_pass(const PassDesc& d, int nstates, int S, int p,
                              const void* in, void* out, uint64_t state_stride,
                              const double* W, const LayerCoef* coef,
                              double* part, void* probs, void* tab, hipStream_t stream);
// Gradient passes on 13-qubit register tiles (complex64).  The checkpoint
// pass (first or middle shape) stores its output with every mixer scalar
// applied; the backward shapes are 0 = seed (the last forward pass fused with
// its adjoint), 1 = middle, 2 = first.
hipError_t launch_fwd13_ckpt_pass(const PassDesc& d, int nstates, int S, int p, const void* in,
                                  void* out, uint64_t stride, const double* W,
                                  const LayerCoef* coef, void* tab, hipStream_t stream);
hipError_t launch_bwd13_pass(const PassDesc& d, int shape, int nstates, int S, int p,
                             const void* psi, void* lam, uint64_t stride, const double* W,
                             const LayerCoef* coef, double* part, int rec_base, int nrec,
                             void* tab, hipStream_t stream);
// Gradient passes on 12-qubit register tiles (complex128), as the 13-qubit
// complex64 ones: 13 <= n <= 22, kind-2 sets with 2 low bits.
hipError_t launch_fwd12_ckpt_pass(const PassDesc& d, int nstates, int S, int p, const void* in,
                                  void* out, uint64_t stride, const double* W,
                                  const LayerCoef* coef, void* tab, hipStream_t stream);
hipError_t launch_bwd12_pass(const PassDesc& d, int shape, int nstates, int S, int p,
                             const void* psi, void* lam, uint64_t stride, const double* W,
                             const LayerCoef* coef, double* part, int rec_base, int nrec,
                             void* tab, hipStream_t stream);

// ---- launchers (kernels.hip) ---------------------------------------------
// prec: 0 = complex128, 1 = complex64.
hipError_t launch_prep(int nprob, int n, const double* Q, double* W,
                       int nstates, int p, const double* gammas,
                       const double* betas, LayerCoef* coef,
                       hipStream_t stream);

// Whole-state evaluation (small.hip): the fold of Q, the p layers, <C> and
// the norm, and the optional probabilities and state, in one launch of one
// work-group per state, for n up to small_fwd_nmax(prec); the adjoint
// gradient likewise up to small_grad_nmax(prec) (prec as QAOA_C64 / C128).
inline int small_fwd_nmax(int prec) { return prec == 1 ? 14 : 13; }
inline int small_grad_nmax(int prec) { return prec == 1 ? 13 : 12; }
hipError_t launch_small_expect(int prec, int n, int p, int S, int nstates, const double* Q,
                               const double* gammas, const double* betas, double* expect,
                               double* norm, void* probs, void* psi, hipStream_t stream);
// The adjoint gradient of the same states (expect nullable), one launch.
hipError_t launch_small_grad(int prec, int n, int p, int S, int nstates, const double* Q,
                             const double* gammas, const double* betas, double* expect,
                             double* dgamma, double* dbeta, hipStream_t stream);
hipError_t launch_fwd_pass(int prec, const PassDesc& d, int nstates, int S,
                           int p, const void* in, void* out,
                           uint64_t state_stride, const double* W,
                           const LayerCoef* coef, double* part, void* probs,
                           hipStream_t stream);

// Sums `nq` partial quantities over `nrec` records for every state in a fixed
// order: part[st][rec][nq].  Quantity q lands in map m with q0[m] <= q <
// q0[m] + cnt[m], at ptr[m][st * cnt[m] + q - q0[m]] (up to 4 maps).
hipError_t launch_reduce_parts(int nstates, int nrec, int nq,
                               const double* part, double* const* out,
                               const int* q0, const int* cnt, int nmap,
                               hipStream_t stream);

// Adjoint pass: records [2p + 2] = (dgamma[p], dbeta[p], <C>, norm) per tile,
// written at part[st][rec_base + tile] of `nrec` records per state.
hipError_t launch_bwd_pass(int prec, const PassDesc& d, int nstates, int S,
                           int p, const void* psi_in, void* lam,
                           uint64_t state_stride, const double* W,
                           const LayerCoef* coef, double* part, int rec_base,
                           int nrec, hipStream_t stream);

// Sampling from probabilities `probs` [nstates][2^n] (state precision):
// scratch bsum/bcdf of sample_scratch_doubles(n, nstates)/2 doubles each.
// With seeds == NULL shot s of state st uses SplitMix64 counter st*shots + s
// of `seed`; otherwise counter s of seeds[st].
hipError_t launch_sample(int prec, int n, int nstates, const void* probs,
                         double* bsum, double* bcdf, int shots, uint64_t seed,
                         const uint64_t* seeds, const double* W, int S, uint64_t* z,
                         double* cz,
                         uint64_t* best_z, double* best_c,
                         hipStream_t stream);
size_t sample_scratch_doubles(int n, int nstates);

// Adam on (gamma, beta) of nb batch entries stored at slots idx[i] (idx NULL:
// slot i): theta [slot][p] each, moments m/v [slot][2p], gradients dgamma/
// dbeta [i][p]; t[slot] counts the steps taken (incremented here).
hipError_t launch_adam(int nb, int p, const int* idx, double* gammas,
                       double* betas, double* m, double* v, const double* dgamma,
                       const double* dbeta, int* t, double lr, double b1,
                       double b2, double eps, hipStream_t stream);

// Batch entry i <- slot idx[i]: Q [n][n] (slot stride qstride doubles) and
// (gamma, beta) [p] into contiguous Q [nb][n][n], g/b [nb][p].
hipError_t launch_gather(int nb, int n, int p, const int* idx, const double* sQ,
                         int qstride, const double* sG, const double* sB,
                         const uint64_t* sSeed, double* Q, double* g, double* b,
                         uint64_t* seeds, hipStream_t stream);

// ---- host runtime shared by the C ABI and the solve queue (capi.hip) -------

int set_error(int code, const char* fmt, ...);
int hip_error(hipError_t e, const char* what);

// Bump allocation of one scratch block: offsets of 256-byte aligned buffers.
struct Carve {
  std::vector<size_t> off;
  size_t total = 0;
  size_t add(size_t bytes) {
    off.push_back(total);
    total += (bytes + 511) & ~(size_t)255;
    return off.size() - 1;
  }
};

// Scratch layout of one call over B problems x S sets.
enum LayoutOp { OP_EXPECT = 0, OP_SAMPLE = 1, OP_GRAD = 2 };
struct Layout {
  Plan plan;
  int prec = 0, B = 0, n = 0, p = 0, S = 0;
  size_t nstates = 0;
  size_t state_bytes = 0;  // one state
  Carve cv;
  size_t iW = 0, iC = 0, iPart = 0, iState = 0, iLam = 0, iProbs = 0,
         iBsum = 0, iBcdf = 0, iCz = 0, iTab = 0;
  std::vector<size_t> iCk;
  int nrec = 0;
  std::vector<int> rec_base;
  char* at(char* base, size_t idx) const { return base + cv.off[idx]; }
};
int make_layout(int op, int prec, int B, int n, int p, int S, int shots,
                Layout* L);

// Optional timing hook: brackets every state-pass launch with events.
struct PassTimer {
  virtual void begin(hipStream_t s, double bytes) = 0;
  virtual void end(hipStream_t s) = 0;
  virtual ~PassTimer() {}
};

// Queue the full pipelines on `s` using the scratch block `base` laid out by
// make_layout.  Inputs Q [B][n][n], gammas/betas [B][S][p] are device FP64.
int enqueue_expect(const Layout& L, char* base, const double* Q,
                   const double* gammas, const double* betas, double* expect,
                   double* norm, void* probs, void* psi, hipStream_t s,
                   PassTimer* tm);
int enqueue_grad(const Layout& L, char* base, const double* Q,
                 const double* gammas, const double* betas, double* expect,
                 double* dgamma, double* dbeta, hipStream_t s, PassTimer* tm);
int enqueue_sample(const Layout& L, char* base, const double* Q,
                   const double* gammas, const double* betas, int shots,
                   uint64_t seed, const uint64_t* seeds, uint64_t* z, double* cz, uint64_t* best_z,
                   double* best_c, double* expect, hipStream_t s,
                   PassTimer* tm);
int kmax_for(int prec, bool two_tiles);
int cpref_for(int prec);

size_t lds_bytes_fwd(int prec, int k);
size_t lds_bytes_bwd(int prec, int k);

}  // namespace dq
