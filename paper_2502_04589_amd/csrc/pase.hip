// Host runtime and C ABI of libpase: hierarchy setup, the V-cycle, the CG
// solves, the projection onto V_H + span{W}, the small eigenproblem and the
// outer loop (paper Alg. 3, one correction step = Alg. 1).
//
// Basis of the augmented space used for step (c): the columns of
// [P L_B^{-T}, W_perp L^{-T}], where B_H = L_B L_B^T, W_perp is W made
// M-orthogonal to V_H (the vector form of the PRECOND-B factorisation of
// Sec. 4) and W_perp^T M W_perp = L L^T.  The basis is M-orthonormal, so the
// augmented pencil (A_Hh, B_Hh) becomes the standard symmetric matrix
//   T = [[L_B^{-1} A_H L_B^{-T},  L_B^{-1} P^T A W_perp L^{-T}],
//        [        (sym)        ,  L^{-1} W_perp^T A W_perp L^{-T}]]
// whose k smallest eigenpairs are the Ritz pairs of V_H + span{W}.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

#include "internal.hpp"

using namespace pase;

namespace {

thread_local std::string g_last_error;

struct Bump {
  char* base;
  size_t off = 0;
  explicit Bump(void* b) : base((char*)b) {}
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T* p = base ? (T*)(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

// Dense symmetric eigensolver for the k smallest pairs: the one-workgroup / cooperative-LDS
// solver up to n = 512, the grid solver in global memory above.
constexpr int kDenseSmallN = 512;
size_t syev_any_work(int n, int k) {
  return n <= kDenseSmallN ? syev_work_doubles(n, k) : syev_large_work_doubles(n, k);
}
void syev_any(int n, int k, double* T, double* w, double* V, double* work, int* info, hipStream_t s) {
  if (n <= kDenseSmallN) launch_syev_lowest(n, k, T, w, V, work, info, s);
  else launch_syev_large(n, k, T, w, V, work, info, s);
}

}  // namespace

void pase::set_last_error(const std::string& msg) { g_last_error = msg; }

struct pase_handle {
  pase_problem prob{};
  pase_options opt{};
  hipStream_t stream = nullptr;
  int dim = 0, L = 0, NS = 0, K = 0;    // L = index of the coarsest level
  Level lev[PASE_MAX_LEVELS];
  // fine multi-vectors (N0 x K)
  double *U = nullptr, *X = nullptr, *R = nullptr, *Z = nullptr, *P = nullptr, *Q = nullptr;
  double *W2 = nullptr, *W3 = nullptr;
  // V-cycle buffers per level (level 0 uses xa and r only)
  double *vb[PASE_MAX_LEVELS] = {}, *vx[PASE_MAX_LEVELS] = {}, *vxa[PASE_MAX_LEVELS] = {}, *vr[PASE_MAX_LEVELS] = {};
  double* kappa = nullptr;
  bool kappa_is_one = false;    // problem given with kappa = NULL (constant coefficient)
  bool fine_general = false;    // tensor-coefficient problem: the fine operator is an assembled stencil
  bool alg = false;             // algebraic input: every level operator and transfer is a CSR matrix
  pase_hierarchy_csr csr{};
  // coarse dense (NH x NH)
  double *AinvL = nullptr, *LBinv = nullptr, *BHinv = nullptr, *C0 = nullptr, *dtmp = nullptr;
  // small problem
  int nT = 0;
  double *Tm = nullptr, *Vs = nullptr, *syw = nullptr;
  double *ca = nullptr, *cb = nullptr, *cc = nullptr;     // NH x K
  double *kk1 = nullptr, *kk2 = nullptr, *kk3 = nullptr, *kk4 = nullptr, *kk5 = nullptr;   // K x K
  // column scalars
  double *lam = nullptr, *rho = nullptr, *rho2 = nullptr, *pq = nullptr, *alpha = nullptr, *beta = nullptr;
  double* sums = nullptr;       // 3K
  double* partial = nullptr;
  size_t partial_doubles = 0;
  int* info = nullptr;          // device status words
  double* zero16 = nullptr;     // 64 zero bytes
  double* setup_scratch = nullptr;
  // mixed precision: FP32 multi-vectors for the correction-form CG and its V-cycle
  float *R32 = nullptr, *Z32 = nullptr, *P32 = nullptr, *Q32 = nullptr, *E32 = nullptr;
  float *vb32[PASE_MAX_LEVELS] = {}, *vx32[PASE_MAX_LEVELS] = {}, *vxa32[PASE_MAX_LEVELS] = {},
        *vr32[PASE_MAX_LEVELS] = {};
  float* AinvL32 = nullptr;
  // structured augmented eigenproblem: C0 = Phi diag(theta) Phi^T, Psi = L_B^{-T} Phi
  bool fast = false;
  bool fast_big = false;        // large coarse space or k > 64: the structured kernels of small_big.hip
  double* sbig = nullptr;       // their per-pair work vectors (2 (N_H + K) x K)
  double *theta = nullptr, *Psi = nullptr, *Gtl = nullptr, *Vtf = nullptr, *Vtf2 = nullptr, *Gf = nullptr;
  double *rqf = nullptr, *resf = nullptr;
  double *cmw = nullptr, *kkb = nullptr, *X0f = nullptr;   // P^T M W, beta, start block
  // complement coordinates c = B_H^{-1} P^T M W of the last projection, kept for the prolongation when
  // W_perp = W - P c was not formed on the fine grid (w_perp false)
  double* cperp = nullptr;
  bool w_perp = true;
  int *permf = nullptr, *statf = nullptr;
  double small_scale = 1.0;
  // learned form: attached network, node log kappa, flexible-PCG column state
  pase_unet* net = nullptr;
  double *logk = nullptr, *rr0 = nullptr, *rr1 = nullptr, *rzo = nullptr;
  int* netmask = nullptr;
  int fallbacks = 0;            // column switches to the V-cycle (this solve)
  int fast_hits = 0;            // corrections solved by the structured path (this solve)
  int last_path = 0;            // 1 accepted, 2 accepted on the wanted pairs' count, 0 dense only,
                                // -1 residual, -2 count, -3 orthonormalisation
  int nev_cur = 0;              // wanted pairs of the running solve (the block minus the guard pairs)
  bool spec = false;            // a structured solution was enqueued and its status is not read yet
  bool retried = false;         // this correction's structured path already restarted from the reduced
                                // Rayleigh-Ritz block
  bool try_fast = true;         // attempt the structured path in this correction
  // mixed form: the projection runs on FP32 vectors with split-BF16 Grams until the residual drops
  // below 1e-6 or stops halving over two corrections (then FP64 to the end of the solve)
  bool proj_lp = false;
  int proj_lp_iters = 0;
  // soft locking: the next correction's fine solves run for the ka columns lock_idx[0..ka); lock_idx[K + j]
  // is the position of column j among them (-1: locked)
  int* lock_idx = nullptr;
  int ka = 0;
  std::vector<int> lock_host;
  // structured small solver: residual acceptance relative to max|theta|, per position of the
  // ascending order (host copy set per correction, device copy small_tolv)
  double small_acc = 1e-11;
  std::vector<double> tolv_host;
  std::vector<double> outer_res;    // the outer residuals of the pairs before this correction
  double* small_tolv = nullptr;
  bool tolv_on = false;
  int fine_cols = 0;
  // PRECOND-A and GCG_AUG (small_solver 2): V_H = level gc (gNH nodes), augmented blocks of
  // gNH + k rows (the coarse coordinates, then the k fine directions)
  bool gcg = false;
  bool psi_only = false;            // the coarse start's eigenbasis without the structured path
  int gc = 0;
  long long gNH = 0;
  double *g_a = nullptr, *g_ahat = nullptr, *g_at = nullptr, *g_bt = nullptr;   // gNH x K
  double *g_alt = nullptr, *g_bet = nullptr, *g_alinv = nullptr;               // K x K
  double *gX = nullptr, *gAX = nullptr, *gBX = nullptr, *gXn = nullptr, *gAXn = nullptr, *gBXn = nullptr;
  double *gP = nullptr, *gBP = nullptr, *gPn = nullptr, *gBPn = nullptr;
  double *gY = nullptr, *gAY = nullptr, *gBY = nullptr, *gY2 = nullptr;
  double *gW = nullptr, *gAW = nullptr, *gBW = nullptr;
  double *gR = nullptr, *gZ = nullptr, *gPp = nullptr, *gQ = nullptr;
  double *gS = nullptr, *gG = nullptr, *gLi = nullptr, *gH = nullptr, *gC = nullptr, *gCJ = nullptr;
  double *gGxx = nullptr, *gGxy = nullptr, *gGyy = nullptr, *gw = nullptr, *glam = nullptr, *glamn = nullptr;
  double *gsyw = nullptr, *gchs = nullptr, *gpart = nullptr, *gnorm = nullptr;
  int* gidx = nullptr;
  // batch scheme (Alg. 7): the composite pairs nearest the shift (bnsel at most), their
  // coordinates along span(u_hat), the selection, and P^T M W before the complement
  int bnsel = 0;
  double *bVw = nullptr, *blw = nullptr, *bZ = nullptr, *bS = nullptr, *bY = nullptr, *bGZ = nullptr;
  double *bmw = nullptr, *bsyw = nullptr;
  int* bsel = nullptr;
  int aug_iters = 0;                // GCG_AUG iterations of this solve
  int aug_restarts = 0;             // ... and its iterations redone after a breakdown
  double* pin_gnorm = nullptr;      // pinned: 2 K column norms
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // per-phase device time of a solve: marks (event, phase) enqueued on the stream and resolved after
  // each synchronisation of the outer loop; a mark of phase -1 opens an interval that is not counted
  // (the stream idles while the host reads the residuals)
  static constexpr int kMarks = 24;
  hipEvent_t evm[kMarks] = {};
  int mark_phase[kMarks] = {};
  int nmark = 0;
  bool timing = false;
  double t_phase[PASE_PHASES] = {};
  // pinned host staging of the per-correction transfers (column sums, Ritz values, status words,
  // locking indices, acceptance factors): truly asynchronous copies, one synchronisation each
  void* pin = nullptr;
  double *pin_sums = nullptr, *pin_lam = nullptr, *pin_tolv = nullptr;
  int *pin_info = nullptr, *pin_st = nullptr, *pin_idx = nullptr;
  std::string err;
};

namespace {

// Phases of the per-phase timers (pase_report.t_phase_ms)
enum Phase { PH_START = 0, PH_RESIDUAL = 1, PH_FINE = 2, PH_PROJECTION = 3, PH_SMALL = 4, PH_PROLONG = 5 };

// Time from the previous mark on is charged to the previous mark's phase; nothing when not timing.
// The outer loop settles every completed interval after each synchronisation.
void settle_marks(pase_handle* h) {
  for (int i = 0; i + 1 < h->nmark; ++i) {
    if (h->mark_phase[i] < 0) continue;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, h->evm[i], h->evm[i + 1]) == hipSuccess) h->t_phase[h->mark_phase[i]] += ms;
  }
  if (h->nmark > 1) {
    std::swap(h->evm[0], h->evm[h->nmark - 1]);
    h->mark_phase[0] = h->mark_phase[h->nmark - 1];
    h->nmark = 1;
  }
}

void mark(pase_handle* h, int phase) {
  if (!h->timing) return;
  if (h->nmark == pase_handle::kMarks) {   // not reached by the outer loop (at most 12 per correction)
    (void)hipStreamSynchronize(h->stream);
    settle_marks(h);
  }
  if (hipEventRecord(h->evm[h->nmark], h->stream) == hipSuccess) h->mark_phase[h->nmark++] = phase;
}

pase_status fail(pase_handle* h, pase_status s, const std::string& msg) {
  if (h) h->err = msg;
  g_last_error = msg;
  return s;
}

#define HIPC(call)                                                                        \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(h, PASE_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_));     \
  } while (0)

long long level_nodes(int dim, int n) {
  long long m = n - 1;
  return dim == 3 ? m * m * m : m * m;
}

bool csr_ok(const pase_csr& c, int rows, int cols) {
  return c.rows == rows && c.cols == cols && rows >= 1 && c.rowptr && c.colind && c.val;
}

// Algebraic input: consistent shapes, every pointer given
pase_status check_csr(const pase_hierarchy_csr* c) {
  if (c->nlevels < 2 || c->nlevels > PASE_MAX_LEVELS) return PASE_E_ARG;
  for (int l = 0; l < c->nlevels; ++l) {
    const int n = c->A[l].rows;
    if (!csr_ok(c->A[l], n, n) || !csr_ok(c->M[l], n, n)) return PASE_E_ARG;
    if (l > 0) {
      const int nf = c->A[l - 1].rows;
      if (!csr_ok(c->P[l], nf, n) || !csr_ok(c->R[l], n, nf)) return PASE_E_ARG;
    }
  }
  return PASE_OK;
}

// level sizes of a problem (grid or algebraic); dim = 0 for algebraic input
void set_levels(pase_handle* h, const pase_problem* prob) {
  if (prob->csr) {
    h->alg = true;
    h->csr = *prob->csr;
    h->dim = 0;
    h->L = prob->csr->nlevels - 1;
    h->NS = 0;
    for (int l = 0; l <= h->L; ++l) {
      h->lev[l].n = h->lev[l].m = 0;
      h->lev[l].N = prob->csr->A[l].rows;
      h->lev[l].h = 0.0;
    }
    return;
  }
  h->dim = prob->dim;
  h->L = prob->nlevels - 1;
  h->NS = prob->dim == 3 ? 27 : 9;
  for (int l = 0; l < prob->nlevels; ++l) {
    h->lev[l].n = prob->n[l];
    h->lev[l].m = prob->n[l] - 1;
    h->lev[l].N = level_nodes(prob->dim, prob->n[l]);
    h->lev[l].h = 1.0 / prob->n[l];
  }
}

pase_status check_problem(const pase_problem* p, const pase_options* o) {
  if (!p || !o) return PASE_E_ARG;
  const int nlev = p->csr ? p->csr->nlevels : p->nlevels;
  if (p->csr) {
    if (p->kappa || p->tensor || p->reaction) return PASE_E_ARG;
    const pase_status st = check_csr(p->csr);
    if (st) return st;
    if (o->precision == PASE_PREC_LEARNED) return PASE_E_UNSUPPORTED;   // the network works on a grid
  } else {
    if (p->dim != 2 && p->dim != 3) return PASE_E_ARG;
    if (p->nlevels < 2 || p->nlevels > PASE_MAX_LEVELS) return PASE_E_ARG;
    for (int l = 0; l < p->nlevels; ++l) {
      if (p->n[l] < 2) return PASE_E_ARG;
      if (l > 0 && p->n[l - 1] != 2 * p->n[l]) return PASE_E_ARG;
    }
  }
  if (o->nev_max < 1 || o->nev_max > PASE_MAX_NEV) return PASE_E_ARG;
  if (o->cg_steps < 1 || o->max_outer < 0 || o->nu < 1) return PASE_E_ARG;
  if (!(o->omega > 0.0)) return PASE_E_ARG;
  if (o->small_solver < 0 || o->small_solver > 2) return PASE_E_ARG;
  if (o->coarse_level < 0 || o->coarse_level >= nlev) return PASE_E_ARG;
  if (!(o->aug_rtol >= 0.0)) return PASE_E_ARG;
  if (o->coarse_level != 0 && o->coarse_level != nlev - 1 && o->small_solver != 2)
    return PASE_E_UNSUPPORTED;   // V_H below the coarsest level: GCG_AUG only
  if (o->locking != 0 && o->locking != 1) return PASE_E_ARG;
  if (o->guard < 0 || o->guard > 64 || o->nev_max + o->guard > PASE_MAX_NEV) return PASE_E_ARG;
  if (o->start != 0 && o->start != 1) return PASE_E_ARG;
  if (!(o->fallback_ratio > 0.0)) return PASE_E_ARG;
  if (o->precision != PASE_PREC_FP64 && o->precision != PASE_PREC_MIXED && o->precision != PASE_PREC_LEARNED)
    return PASE_E_UNSUPPORTED;
  if (o->precision == PASE_PREC_LEARNED && p->dim != 3 && !p->csr) return PASE_E_UNSUPPORTED;   // the network is 3D
  if (!p->csr && p->tensor && (p->dim != 3 || p->kappa)) return PASE_E_ARG;
  if (!p->tensor && p->reaction) return PASE_E_ARG;
  if (p->tensor && o->precision == PASE_PREC_LEARNED) return PASE_E_UNSUPPORTED;   // the network reads log kappa
  return PASE_OK;
}

// Lays out the workspace; with base == nullptr only counts bytes.
size_t layout(pase_handle* h, void* base) {
  Bump b(base);
  const int dim = h->dim;
  const long long N0 = h->lev[0].N;
  const size_t K = h->K;
  const size_t NS = h->NS;
  const size_t mv = (size_t)N0 * K;
  const size_t NHs = (size_t)h->lev[h->L].N;
  // fine multi-vectors; setup reuses this block as scratch (Galerkin probes, then an N_H x N_H
  // product and the blocked factorisations of the coarse matrices)
  const size_t coarse_setup = NHs * NHs + std::max(cholesky_large_scratch_doubles((int)NHs),
                                                   trinv_large_scratch_doubles((int)NHs)) + 64;
  const size_t fine_doubles = std::max({10 * mv, 3 * (size_t)N0 * NS + 64, coarse_setup});
  double* fine = b.take<double>(fine_doubles);
  h->setup_scratch = fine;
  double* f = fine;
  auto nxt = [&](size_t n) { double* r = f; if (f) f += n; return r; };
  h->U = nxt(mv); h->X = nxt(mv); h->R = nxt(mv); h->Z = nxt(mv); h->P = nxt(mv); h->Q = nxt(mv);
  h->W2 = nxt(mv); h->W3 = nxt(mv);
  h->vxa[0] = nxt(mv); h->vr[0] = nxt(mv);
  const long long ne = (long long)h->lev[0].n * h->lev[0].n * (dim == 3 ? h->lev[0].n : 1);
  h->kappa = b.take<double>((size_t)ne);
  h->lev[0].dinv = b.take<double>((size_t)N0);
  if (h->fine_general) h->lev[0].coef = b.take<double>((size_t)N0 * h->NS);
  for (int l = 1; l <= h->L; ++l) {
    const size_t Nl = (size_t)h->lev[l].N;
    h->lev[l].coef = b.take<double>(Nl * NS);
    h->lev[l].dinv = b.take<double>(Nl);
    h->vb[l] = b.take<double>(Nl * K);
    h->vx[l] = b.take<double>(Nl * K);
    h->vxa[l] = b.take<double>(Nl * K);
    h->vr[l] = b.take<double>(Nl * K);
  }
  if (h->opt.precision == PASE_PREC_MIXED) {
    h->R32 = b.take<float>(mv); h->Z32 = b.take<float>(mv); h->P32 = b.take<float>(mv);
    h->Q32 = b.take<float>(mv); h->E32 = b.take<float>(mv);
    h->vxa32[0] = b.take<float>(mv); h->vr32[0] = b.take<float>(mv);
    for (int l = 1; l <= h->L; ++l) {
      const size_t Nl = (size_t)h->lev[l].N;
      h->vb32[l] = b.take<float>(Nl * K); h->vx32[l] = b.take<float>(Nl * K);
      h->vxa32[l] = b.take<float>(Nl * K); h->vr32[l] = b.take<float>(Nl * K);
    }
    const size_t NHf = (size_t)h->lev[h->L].N;
    h->AinvL32 = b.take<float>(NHf * NHf);
  }
  h->lock_idx = b.take<int>(2 * K);
  h->small_tolv = b.take<double>(K);
  if (h->opt.precision == PASE_PREC_LEARNED) {
    h->logk = b.take<double>((size_t)N0);
    h->rr0 = b.take<double>(K); h->rr1 = b.take<double>(K); h->rzo = b.take<double>(K);
    h->netmask = b.take<int>(K);
  }
  const size_t NH = (size_t)h->lev[h->L].N;
  h->AinvL = b.take<double>(NH * NH);
  h->LBinv = b.take<double>(NH * NH);
  h->BHinv = b.take<double>(NH * NH);
  h->C0 = b.take<double>(NH * NH);
  h->dtmp = b.take<double>(NH * NH);
  h->nT = (int)(NH + K);
  const size_t nT = (size_t)h->nT;
  h->gcg = (h->opt.small_solver == 2);
  h->gc = (h->opt.coarse_level > 0) ? h->opt.coarse_level : h->L;
  h->gNH = h->lev[h->gc].N;
  h->psi_only = h->gcg && h->opt.start == 1 && (int)NH <= syev_large_max_n();
  if (h->psi_only) {
    // the coarse start's eigenbasis of the coarsest level (the augmented problems go to GCG_AUG)
    h->Tm = b.take<double>(NH * NH);
    h->syw = b.take<double>(syev_any_work((int)NH, (int)NH));
    h->theta = b.take<double>(NH);
    h->Psi = b.take<double>(NH * NH);
  }
  if (h->gcg) {
    const size_t gN = (size_t)h->gNH, Na = gN + K, K2 = 2 * K, K3 = 3 * K;
    h->g_a = b.take<double>(gN * K); h->g_ahat = b.take<double>(gN * K);
    h->g_at = b.take<double>(gN * K); h->g_bt = b.take<double>(gN * K);
    h->g_alt = b.take<double>(K * K); h->g_bet = b.take<double>(K * K); h->g_alinv = b.take<double>(K * K);
    double** nk[] = {&h->gX, &h->gAX, &h->gBX, &h->gXn, &h->gAXn, &h->gBXn, &h->gP, &h->gBP, &h->gPn, &h->gBPn,
                     &h->gW, &h->gAW, &h->gBW, &h->gR, &h->gZ, &h->gPp, &h->gQ};
    for (double** q : nk) *q = b.take<double>(Na * K);
    double** n2k[] = {&h->gY, &h->gAY, &h->gBY, &h->gY2};
    for (double** q : n2k) *q = b.take<double>(Na * K2);
    h->gS = b.take<double>(K * K2); h->gG = b.take<double>(K2 * K2); h->gLi = b.take<double>(K2 * K2);
    h->gH = b.take<double>(K3 * K3); h->gC = b.take<double>(K3 * K); h->gCJ = b.take<double>(K2 * K);
    h->gGxx = b.take<double>(K * K); h->gGxy = b.take<double>(K * K2); h->gGyy = b.take<double>(K2 * K2);
    h->gw = b.take<double>(K3); h->glam = b.take<double>(K); h->glamn = b.take<double>(K);
    // Rayleigh-Ritz sizes run from K to 3K: the largest work of each eigensolver branch
    h->gsyw = b.take<double>(std::max(syev_any_work((int)std::min<size_t>(K3, kDenseSmallN), (int)K),
                                      syev_any_work((int)K3, (int)K)));
    h->gchs = b.take<double>(std::max(cholesky_large_scratch_doubles((int)K2), trinv_large_scratch_doubles((int)K2)));
    h->gpart = b.take<double>(std::max(gram_tn_partial_doubles((long long)Na, (int)K2, (int)K2),
                                       gram_tn_partial_doubles((long long)Na, (int)K, (int)K2)));
    h->gnorm = b.take<double>(2 * K);
    h->gidx = b.take<int>(K);
  }
  if (!h->gcg && h->nT <= syev_large_max_n() && (int)K <= syev_max_k()) {
    const bool fit_small = (int)K <= small_fast_max_k() && (int)NH <= small_fast_max_nh();
    const bool fit_big = (int)K <= small_big_max_k() && (int)NH <= small_big_max_nh();
    h->fast = (h->opt.small_solver == 0) && (fit_small || fit_big);
    h->fast_big = h->fast && !fit_small;
    h->Tm = b.take<double>(nT * nT);
    h->Vs = b.take<double>(nT * K);
    size_t sw = syev_any_work(h->nT, (int)K);
    if (h->fast) sw = std::max(sw, syev_any_work((int)NH, (int)NH));   // setup: all of C0
    h->syw = b.take<double>(sw);
    if (h->fast && 2 * K <= (size_t)batch_select_max()) {
      // batch scheme: up to 2 K composite pairs nearest the shift
      h->bnsel = (int)std::min(2 * K, nT);
      const size_t ns = (size_t)h->bnsel;
      h->bVw = b.take<double>(nT * ns);
      h->blw = b.take<double>(ns);
      h->bZ = b.take<double>(nT * K);
      h->bS = b.take<double>(K * ns);
      h->bY = b.take<double>(K * ns);
      h->bGZ = b.take<double>(K * K);
      h->bmw = b.take<double>(NH * K);
      h->bsyw = b.take<double>(syev_window_work_doubles(h->nT, h->bnsel));
      h->bsel = b.take<int>(K);
    }
  }
  if (h->fast) {
    h->theta = b.take<double>(NH);
    h->Psi = b.take<double>(NH * NH);
    h->Gtl = b.take<double>(NH * K);
    h->Vtf = b.take<double>(nT * K);
    h->Vtf2 = b.take<double>(nT * K);
    h->Gf = b.take<double>(K * K);
    h->rqf = b.take<double>(K);
    h->resf = b.take<double>(K);
    h->cmw = b.take<double>(NH * K);
    h->kkb = b.take<double>(K * K);
    h->X0f = b.take<double>(nT * K);
    h->permf = b.take<int>(K);
    h->statf = b.take<int>(4);
    if (h->fast_big) h->sbig = b.take<double>(small_big_scratch_doubles((int)NH, (int)K));
  }
  h->ca = b.take<double>(NH * K);
  h->cb = b.take<double>(NH * K);
  h->cc = b.take<double>(NH * K);
  h->cperp = b.take<double>(NH * K);
  h->kk1 = b.take<double>(K * K); h->kk2 = b.take<double>(K * K); h->kk3 = b.take<double>(K * K);
  h->kk4 = b.take<double>(K * K); h->kk5 = b.take<double>(K * K);
  h->lam = b.take<double>(K); h->rho = b.take<double>(K); h->rho2 = b.take<double>(K);
  h->pq = b.take<double>(K); h->alpha = b.take<double>(K); h->beta = b.take<double>(K);
  h->sums = b.take<double>(3 * K);
  // partials: max over coldot, gram and eig-residual reductions for every k <= K
  size_t pd = 0;
  for (int k = 1; k <= (int)K; ++k) {
    pd = std::max(pd, (size_t)coldot_tiles(N0, k) * k);
    pd = std::max(pd, (size_t)2 * gram_tiles(N0, k) * k * k);
    pd = std::max(pd, (size_t)grid_launch(N0, k).blocks * 3 * k);
    if (h->alg) pd = std::max(pd, (size_t)csr_tiles(N0) * 3 * k);
    if (dim == 3) pd = std::max(pd, (size_t)fine3_max_spatial_blocks(h->lev[0].m) * 3 * k);
  }
  h->partial_doubles = pd;
  h->partial = b.take<double>(pd);
  h->info = b.take<int>(16);
  h->zero16 = b.take<double>(8);
  return b.off + 256;
}

// ----------------------------------------------------------------- operators
StencilArgs stencil_args(pase_handle* h, int l, int k) {
  StencilArgs a{};
  const Level& lv = h->lev[l];
  a.dim = h->dim;
  a.m = lv.m;
  a.N = lv.N;
  a.k = k;
  a.h = lv.h;
  a.src = (l == 0 && !h->fine_general) ? ASource::Kappa : ASource::Assembled;
  a.kappa = h->kappa;
  a.coef = lv.coef;
  a.dinv = lv.dinv;
  a.omega = h->opt.omega;
  return a;
}

// Every stencil application goes through here: the 3D fine level uses the
// LDS-staged kernel, 2D problems and coarse levels the generic one.
CsrMat csr_mat(const pase_csr& c);

void stencil_op(pase_handle* h, int l, int k, Epi epi, const void* x, const void* b, void* out1, void* out2,
                int fp32 = 0) {
  if (h->alg) {
    CsrOpArgs a{};
    a.rows = h->lev[l].N;
    a.k = k;
    a.A = csr_mat(h->csr.A[l]);
    a.M = csr_mat(h->csr.M[l]);
    a.dinv = h->lev[l].dinv;
    a.omega = h->opt.omega;
    a.x = x;
    a.b = b;
    a.lam = h->lam;
    a.out1 = out1;
    a.out2 = out2;
    a.partial = h->partial;
    a.fp32 = fp32;
    launch_csr_op(a, epi, h->stream);
    return;
  }
  // 3D: the LDS-tiled stencil on every level.  The fine level reads kappa per element (or the
  // assembled row of the tensor-coefficient problem); kappa = 1 takes the constant stencil on every
  // level (nested Q1 spaces with exact integration: the Galerkin operator P^T A P equals the Q1
  // stencil of the coarse mesh); otherwise a coarse level reads its assembled Galerkin row.  M is the
  // Q1 mass stencil of width h_l on every level, which the Galerkin product of the fine mass equals.
  if (h->dim == 3) {
    const bool coarse_rows = (l > 0 && !h->kappa_is_one);
    Fine3Args f{};
    f.m = h->lev[l].m;
    f.k = k;
    f.h = h->lev[l].h;
    f.kappa = (h->kappa_is_one || h->fine_general || l > 0) ? nullptr : h->kappa;
    f.coef = coarse_rows ? h->lev[l].coef : ((h->fine_general && l == 0) ? h->lev[0].coef : nullptr);
    f.x = x;
    f.b = b;
    f.lam = h->lam;
    f.out1 = out1;
    f.out2 = out2;
    f.partial = h->partial;
    f.omega = h->opt.omega;
    f.nzc = fine3_default_nzc(f.m);
    f.fp32 = fp32;
    f.zero = h->zero16;
    f.dinv = h->lev[l].dinv;
    launch_fine3(f, epi, h->stream);
    return;
  }
  StencilArgs a = stencil_args(h, l, k);
  a.x = x;
  a.b = b;
  a.lam = h->lam;
  a.out1 = out1;
  a.out2 = out2;
  a.partial = h->partial;
  a.fp32 = fp32;
  launch_stencil(a, epi, h->stream);
}

CsrMat csr_mat(const pase_csr& c) { return CsrMat{c.rowptr, c.colind, c.val}; }

// restriction from level l to l + 1 and prolongation from level l to l - 1 ((=, +=, -=) by mode)
void xfer_restrict(pase_handle* h, int l, int k, const void* xf, void* xc, int fp32) {
  if (h->alg) {
    launch_csr_apply(csr_mat(h->csr.R[l + 1]), h->lev[l + 1].N, k, xf, xc, 0, fp32, h->stream);
    return;
  }
  launch_restrict(h->dim, h->lev[l].m, h->lev[l + 1].m, k, xf, xc, fp32, h->stream);
}

void xfer_prolong(pase_handle* h, int l, int k, const void* xc, void* xf, int mode, int fp32) {
  if (h->alg) {
    launch_csr_apply(csr_mat(h->csr.P[l]), h->lev[l - 1].N, k, xc, xf, mode, fp32, h->stream);
    return;
  }
  launch_prolong(h->dim, h->lev[l - 1].m, h->lev[l].m, k, xc, xf, mode, fp32, h->stream);
}

int eigres_tiles(pase_handle* h, int k, bool fp32 = false) {
  if (h->alg) return csr_tiles(h->lev[0].N);
  if (h->dim == 3) return fine3_spatial_blocks(h->lev[0].m, fine3_default_nzc(h->lev[0].m), k, fp32);
  return grid_launch(h->lev[0].N, k).tiles;
}

void apply_AM(pase_handle* h, int l, int k, const double* x, double* ax, double* mx) {
  stencil_op(h, l, k, EPI_AM, x, nullptr, ax, mx);
}

// Buffers of one V-cycle precision.
struct VBufs {
  void* b[PASE_MAX_LEVELS];
  void* x[PASE_MAX_LEVELS];
  void* xa[PASE_MAX_LEVELS];
  void* r[PASE_MAX_LEVELS];
  int fp32;
};

VBufs vbufs(pase_handle* h, int fp32) {
  VBufs v{};
  for (int l = 0; l <= h->L; ++l) {
    v.b[l] = fp32 ? (void*)h->vb32[l] : (void*)h->vb[l];
    v.x[l] = fp32 ? (void*)h->vx32[l] : (void*)h->vx[l];
    v.xa[l] = fp32 ? (void*)h->vxa32[l] : (void*)h->vxa[l];
    v.r[l] = fp32 ? (void*)h->vr32[l] : (void*)h->vr[l];
  }
  v.fp32 = fp32;
  return v;
}

// x = V(b) on level l (x must not alias b), in the precision of B.  With dot (level 0 only),
// dot[j] = b_j^T x_j as well: fused into the last sweep on the 3D path.
void vcycle(pase_handle* h, const VBufs& B, int l, int k, const void* b, void* x, double* dot = nullptr) {
  hipStream_t s = h->stream;
  if (l == h->L) {
    const int NH = (int)h->lev[l].N;
    if (B.fp32)
      launch_gemm_f32(false, false, NH, k, NH, 1.0, h->AinvL32, NH, (const float*)b, k, 0.0, (float*)x, k, s);
    else
      launch_gemm(false, false, NH, k, NH, 1.0, h->AinvL, NH, (const double*)b, k, 0.0, (double*)x, k, s);
    return;
  }
  const Level& lv = h->lev[l];
  void* t0 = B.xa[l];
  void* t1 = x;
  // sweeps alternate t0, t1, t0, ...; the last of the 2 nu sweeps lands in t1 = x
  void* cur = t0;
  void* oth = t1;
  int i0 = 1;
  if (h->dim == 3 && h->kappa_is_one && h->opt.nu >= 2) {
    // constant coefficient: the first two sweeps from x = 0 in one pass over b
    stencil_op(h, l, k, EPI_SWEEP2, b, nullptr, t1, nullptr, B.fp32);
    cur = t1;
    oth = t0;
    i0 = 2;
  } else if (h->dim == 3 && !h->alg && h->opt.nu >= 2) {
    // variable coefficient: the same pass, the first sweep's x1 = omega D^{-1} b formed as the
    // planes of b are staged
    stencil_op(h, l, k, EPI_SWEEP2V, b, b, t1, nullptr, B.fp32);
    cur = t1;
    oth = t0;
    i0 = 2;
  } else if (h->dim == 3 && !h->alg && !h->kappa_is_one && h->opt.nu == 1) {
    // variable coefficient, one sweep: x1 = omega D^{-1} b is never stored; the residual pass
    // forms it as the planes of b are staged, and the prolongation adds it to the correction
    stencil_op(h, l, k, EPI_RESID1V, b, nullptr, B.r[l], nullptr, B.fp32);
    xfer_restrict(h, l, k, B.r[l], B.b[l + 1], B.fp32);
    vcycle(h, B, l + 1, k, B.b[l + 1], B.x[l + 1]);
    launch_prolong_first(h->dim, lv.m, h->lev[l + 1].m, k, B.x[l + 1], cur, b, lv.dinv, h->opt.omega, B.fp32, s);
    i0 = -1;   // pre-smoothing, residual and prolongation done
  } else {
    launch_first_sweep(h->dim, lv.N, k, lv.dinv, h->opt.omega, b, t0, B.fp32, s);
  }
  if (i0 >= 0) {
    for (int i = i0; i < h->opt.nu; ++i) {
      stencil_op(h, l, k, EPI_SWEEP, cur, b, oth, nullptr, B.fp32);
      std::swap(cur, oth);
    }
    stencil_op(h, l, k, EPI_RESID, cur, b, B.r[l], nullptr, B.fp32);
    xfer_restrict(h, l, k, B.r[l], B.b[l + 1], B.fp32);
    vcycle(h, B, l + 1, k, B.b[l + 1], B.x[l + 1]);
    xfer_prolong(h, l + 1, k, B.x[l + 1], cur, 1, B.fp32);
  }
  const bool fuse = dot && l == 0 && h->dim == 3;
  for (int i = 0; i < h->opt.nu; ++i) {
    const bool last = i + 1 == h->opt.nu;
    stencil_op(h, l, k, (fuse && last) ? EPI_SWEEPDOT : EPI_SWEEP, cur, b, oth, nullptr, B.fp32);
    std::swap(cur, oth);
  }
  if (fuse) {
    launch_reduce_partials(eigres_tiles(h, k, B.fp32), k, h->partial, dot, s);
  } else if (dot) {
    if (B.fp32) launch_coldot_f32(lv.N, k, (const float*)b, (const float*)x, h->partial, dot, s);
    else launch_coldot(lv.N, k, (const double*)b, (const double*)x, h->partial, 0, dot, s);
  }
}

void vcycle(pase_handle* h, int l, int k, const double* b, double* x, double* dot = nullptr) {
  vcycle(h, vbufs(h, 0), l, k, b, x, dot);
}

// Q = A P and pq[j] = p_j^T A p_j on level 0 (fused into the stencil on the 3D path)
void apply_dot(pase_handle* h, int k, const void* P, void* Q, double* pq, int fp32) {
  const long long N = h->lev[0].N;
  if (h->dim == 3) {
    stencil_op(h, 0, k, EPI_AMDOT, P, nullptr, Q, nullptr, fp32);
    launch_reduce_partials(eigres_tiles(h, k, fp32), k, h->partial, pq, h->stream);
    return;
  }
  stencil_op(h, 0, k, EPI_AM, P, nullptr, Q, nullptr, fp32);
  if (fp32) launch_coldot_f32(N, k, (const float*)P, (const float*)Q, h->partial, pq, h->stream);
  else launch_coldot(N, k, (const double*)P, (const double*)Q, h->partial, 0, pq, h->stream);
}

// composite restriction: xc (N_L x k) = P^T xf
void restrict_all(pase_handle* h, int k, const double* xf, double* xc) {
  const double* src = xf;
  for (int l = 0; l < h->L; ++l) {
    double* dst = (l + 1 == h->L) ? xc : h->vr[l + 1];
    xfer_restrict(h, l, k, src, dst, 0);
    src = dst;
  }
}

// composite prolongation into the fine level: xf (=, +=, -=) P xc
void prolong_all(pase_handle* h, int k, const double* xc, double* xf, int mode) {
  const double* src = xc;
  for (int l = h->L; l >= 1; --l) {
    double* dst = (l == 1) ? xf : h->vxa[l - 1];
    xfer_prolong(h, l, k, src, dst, (l == 1) ? mode : 0, 0);
    src = dst;
  }
}

void coldot(pase_handle* h, long long N, int k, const double* x, const double* y, double* out) {
  launch_coldot(N, k, x, y, h->partial, 0, out, h->stream);
}

// s PCG steps per column on A x = b from x0 (X0, not modified) into X, with residual
// R = b - A x0 given (overwritten; it is left at the residual of step s - 1, the last step
// updating x only).  p_0 = z_0 by exchanging the Z and P buffers, and the first update reads
// x0 from X0, so neither start needs a copy.
// With pos (two CG steps only): X0 and X are full blocks of leading dimension ldx, column j of them
// solved as column pos[j] of the k-column blocks (R, the residual, is the gathered one) and copied
// from X0 where pos[j] < 0.
void pcg(pase_handle* h, int k, const double* X0, double* X, double* R, const int* pos = nullptr, int ldx = 0) {
  hipStream_t s = h->stream;
  const long long N = h->lev[0].N;
  vcycle(h, 0, k, R, h->Z, h->rho);
  std::swap(h->Z, h->P);
  if (h->opt.cg_steps == 2) {
    // the same two steps with one x update: r1 = r0 - a0 A p0, p1 = z1 + b p0 (formed in Z, so p0
    // stays in P), x = x0 + a0 p0 + a1 p1; a1 goes to the beta vector once b has been used
    apply_dot(h, k, h->P, h->Q, h->pq, 0);
    launch_pcg_alpha(k, h->rho, h->pq, h->alpha, s);
    launch_rsub(N, k, h->alpha, h->Q, R, s);
    vcycle(h, 0, k, R, h->Z, h->rho2);
    launch_pcg_beta(k, h->rho2, h->rho, h->beta, s);
    launch_zadd(N, k, h->beta, h->P, h->Z, s);
    apply_dot(h, k, h->Z, h->Q, h->pq, 0);
    launch_pcg_alpha(k, h->rho2, h->pq, h->beta, s);
    if (pos) launch_axpy3_merge(N, k, ldx, pos, h->alpha, h->P, h->beta, h->Z, X0, X, s);
    else launch_axpy3(N, k, h->alpha, h->P, h->beta, h->Z, X0, X, s);
    return;
  }
  for (int j = 0; j < h->opt.cg_steps; ++j) {
    apply_dot(h, k, h->P, h->Q, h->pq, 0);
    launch_pcg_alpha(k, h->rho, h->pq, h->alpha, s);
    // the last step's residual is not needed (R is scratch to the callers): x update only
    double* Rj = (j + 1 < h->opt.cg_steps) ? R : nullptr;
    if (j == 0 && X0 != X) launch_axpy2_from(N, k, h->alpha, h->P, h->Q, X0, X, Rj, s);
    else launch_axpy2(N, k, h->alpha, h->P, h->Q, X, Rj, s);
    if (j + 1 < h->opt.cg_steps) {
      vcycle(h, 0, k, R, h->Z, h->rho2);
      launch_pcg_beta(k, h->rho2, h->rho, h->beta, s);
      launch_xpby(N, k, h->Z, h->beta, h->P, s);
      std::swap(h->rho, h->rho2);
    }
  }
}

// Mixed precision: s FP32 PCG steps per column on the correction equation A E = R from E = 0
// (R = lam M U - A U, the FP64 residual), then W = U + E in FP64.  In exact arithmetic W equals
// the iterate of s PCG steps on A w = lam M u from w = u.
// With pos: U and W are full blocks of leading dimension ldw, column j of W = U + E[:, pos[j]] (U where
// pos[j] < 0), and R is the gathered k-column residual.
void pcg_correction_f32(pase_handle* h, int k, const double* U, const double* R, double* W, const int* pos = nullptr,
                        int ldw = 0) {
  hipStream_t s = h->stream;
  const long long N = h->lev[0].N;
  const size_t nk = (size_t)N * k;
  const VBufs B = vbufs(h, 1);
  float* r = h->R32;
  launch_cg_start_f32(nk, R, r, h->E32, s);
  vcycle(h, B, 0, k, r, h->Z32, h->rho);
  std::swap(h->Z32, h->P32);                                  // p_0 = z_0
  for (int j = 0; j < h->opt.cg_steps; ++j) {
    apply_dot(h, k, h->P32, h->Q32, h->pq, 1);
    launch_pcg_alpha(k, h->rho, h->pq, h->alpha, s);
    launch_axpy2_f32(N, k, h->alpha, h->P32, h->Q32, h->E32, (j + 1 < h->opt.cg_steps) ? r : nullptr, s);
    if (j + 1 < h->opt.cg_steps) {
      vcycle(h, B, 0, k, r, h->Z32, h->rho2);
      launch_pcg_beta(k, h->rho2, h->rho, h->beta, s);
      launch_xpby_f32(N, k, h->Z32, h->beta, h->P32, s);
      std::swap(h->rho, h->rho2);
    }
  }
  if (pos) launch_add_f2d_merge(N, k, ldw, pos, U, h->E32, W, s);
  else launch_add_f2d(nk, U, h->E32, W, s);
}

// Learned form: z = N(r) for the columns still on the network, z = V(r) for the others.
// non = number of columns on the network (the host copy of the mask count); scratch (N x k)
// holds the network's output while some columns are on the V-cycle.
pase_status learned_precond(pase_handle* h, int k, const double* R, double* Z, int non, double* scratch) {
  hipStream_t s = h->stream;
  const long long N = h->lev[0].N;
  if (non < k) vcycle(h, 0, k, R, Z);
  if (non == 0) return PASE_OK;
  const pase_status st = pase_unet_apply(h->net, k, R, h->logk, (non == k) ? Z : scratch);
  if (st) return fail(h, st, std::string("network: ") + pase_unet_last_error(h->net));
  if (non < k) launch_select_cols(N, k, h->netmask, scratch, Z, s);
  return PASE_OK;
}

// s steps of flexible PCG per column on A x = b from x (in X), R = b - A x given, preconditioned
// by the network; beta_j = r_{j+1}^T (z_{j+1} - z_j) / (r_j^T z_j) (Notay's flexible CG).  A
// column whose residual norm does not fall below half its previous value switches to the
// V-cycle for the remaining steps; the step is kept and the recurrence restarts (beta = 0), so
// the remaining steps are V-cycle PCG from that iterate.  Returns the number of switches.
pase_status learned_pcg(pase_handle* h, int k, const double* X0, double* X, double* R, int* switches,
                        double* scratch) {
  hipStream_t s = h->stream;
  const long long N = h->lev[0].N;
  *switches = 0;
  launch_fill_int(k, 1, h->netmask, s);
  int non = k;
  std::vector<int> mk(k);
  pase_status st = learned_precond(h, k, R, h->Z, non, scratch);
  if (st) return st;
  std::swap(h->Z, h->P);                                      // p_0 = z_0
  coldot(h, N, k, R, h->P, h->rho);
  for (int j = 0; j < h->opt.cg_steps; ++j) {
    apply_AM(h, 0, k, h->P, h->Q, nullptr);
    coldot(h, N, k, h->P, h->Q, h->pq);
    launch_pcg_alpha(k, h->rho, h->pq, h->alpha, s);
    if (non > 0) coldot(h, N, k, R, R, h->rr0);
    if (j == 0 && X0 != X) launch_axpy2_from(N, k, h->alpha, h->P, h->Q, X0, X, R, s);
    else launch_axpy2(N, k, h->alpha, h->P, h->Q, X, R, s);
    if (non > 0) {
      coldot(h, N, k, R, R, h->rr1);
      launch_fallback(k, h->opt.fallback_ratio, h->rr1, h->rr0, h->netmask, s);
    }
    if (j + 1 < h->opt.cg_steps) {
      if (non > 0) {
        HIPC(hipMemcpyAsync(mk.data(), h->netmask, sizeof(int) * k, hipMemcpyDeviceToHost, s));
        HIPC(hipStreamSynchronize(s));
        int c = 0;
        for (int v : mk) c += (v == 1);
        *switches += non - c;
        non = c;
      }
      coldot(h, N, k, R, (j == 0) ? h->P : h->Z, h->rzo);     // r_{j+1}^T z_j (p_0 = z_0)
      st = learned_precond(h, k, R, h->Z, non, scratch);
      if (st) return st;
      coldot(h, N, k, R, h->Z, h->rho2);                      // r_{j+1}^T z_{j+1}
      launch_flex_beta(k, h->rho2, h->rzo, h->rho, h->netmask, h->beta, s);
      launch_xpby(N, k, h->Z, h->beta, h->P, s);
      std::swap(h->rho, h->rho2);
    }
  }
  if (non > 0) {
    HIPC(hipMemcpyAsync(mk.data(), h->netmask, sizeof(int) * k, hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    int c = 0;
    for (int v : mk) c += (v == 1);
    *switches += non - c;
  }
  return PASE_OK;
}

// R = lam M U - A U with fused column sums (|R|^2, |MU|^2, U.MU) into h->sums
void eig_residual(pase_handle* h, int k, const double* U, double* R) {
  stencil_op(h, 0, k, EPI_EIGRES, U, nullptr, R, nullptr);
  launch_reduce_partials(eigres_tiles(h, k), 3 * k, h->partial, h->sums, h->stream);
}

// Cholesky-QR in the M inner product: U <- U L^{-T}, U^T M U = L L^T.  info slot 'slot'.
void cholqr_m(pase_handle* h, int k, double*& U, double*& spare, int slot) {
  hipStream_t s = h->stream;
  const long long N = h->lev[0].N;
  apply_AM(h, 0, k, U, nullptr, h->W3);
  launch_gram2_sym(N, k, U, h->W3, nullptr, h->partial, gram_tiles(N, k), h->kk2, nullptr, s);
  launch_cholinv(k, h->kk2, h->info + slot, s);            // kk2 <- L^{-1}
  launch_tsmm(N, k, U, h->kk2, spare, 0, 1, s);
  std::swap(U, spare);
}

// U = P y_H + W_perp y_W from the small problem's vectors in Vs (y_W = Li^T V_W) and y_H given (y_H is
// overwritten).  When W_perp = W - P c was not formed, U = P (y_H - c y_W) + W y_W.
void prolongation_tail(pase_handle* h, int k, double* yH) {
  hipStream_t s = h->stream;
  const long long N = h->lev[0].N;
  const int NH = (int)h->lev[h->L].N;
  launch_gemm(true, false, k, k, k, 1.0, h->kk3, k, h->Vs + (size_t)NH * k, k, 0.0, h->kk4, k, s);
  if (!h->w_perp) launch_gemm(false, false, NH, k, k, -1.0, h->cperp, k, h->kk4, k, 1.0, yH, k, s);
  prolong_all(h, k, yH, h->U, 0);
  launch_tsmm(N, k, h->X, h->kk4, h->U, 1, 0, s);
}

// Dense path of the small problem, then the prolongation: G = LB^{-1} a Li^T, T = [[C0, G], [G^T, H]].
pase_status correction_dense_tail(pase_handle* h, int k) {
  hipStream_t s = h->stream;
  const int NH = (int)h->lev[h->L].N;
  const int nT = NH + k;
  mark(h, PH_SMALL);
  launch_gemm(false, false, NH, k, NH, 1.0, h->LBinv, NH, h->ca, k, 0.0, h->cb, k, s);
  launch_gemm(false, true, NH, k, k, 1.0, h->cb, k, h->kk3, k, 0.0, h->cc, k, s);
  launch_set_diag_block(nT, NH, k, h->C0, h->cc, h->kk5, h->Tm, s);
  syev_any(nT, k, h->Tm, h->lam, h->Vs, h->syw, h->info + 2, s);
  mark(h, PH_PROLONG);
  launch_gemm(true, false, NH, k, NH, 1.0, h->LBinv, NH, h->Vs, k, 0.0, h->cb, k, s);   // y_H
  prolongation_tail(h, k, h->cb);
  return PASE_OK;
}

// The structured small solver from the start block in X0f (Gt, H = kk5 and Li = kk3 formed),
// its certification, and the speculative prolongation of its solution: y_H into cc (so that a and
// its restriction in ca stay for the dense path); the caller reads statf with its next
// synchronisation (correction_resolve).
void structured_attempt(pase_handle* h, int k) {
  hipStream_t s = h->stream;
  const int NH = (int)h->lev[h->L].N;
  const int nT = NH + k;
  const double sc = h->small_scale;
  const double* tv = h->tolv_on ? h->small_tolv : nullptr;
  const int nevc = (h->nev_cur >= 1 && h->nev_cur <= k) ? h->nev_cur : k;
  if (h->fast_big) {
    launch_small_rqi_big(NH, k, h->theta, h->Gtl, h->kk5, h->lam, h->X0f, sc, tv, h->Vtf, h->rqf, h->sbig, s);
    launch_vorth2(nT, k, h->Vtf, h->Vtf2, h->Gf, h->statf + 2, s);
    launch_small_rr_big(NH, k, h->theta, h->Gtl, h->kk5, h->Vtf, h->rqf, h->resf, h->sbig, s);
    launch_small_accept_big(NH, k, nevc, h->theta, h->Gtl, h->kk5, h->rqf, h->resf, h->small_acc * sc, tv, 1e-9 * sc,
                            h->lam, h->permf, h->statf, h->sbig, s);
  } else {
    launch_small_rqi(NH, k, h->theta, h->Gtl, h->kk5, h->lam, h->X0f, sc, tv, h->Vtf, h->rqf, s);
    launch_vorth2(nT, k, h->Vtf, h->Vtf2, h->Gf, h->statf + 2, s);
    launch_small_rr(NH, k, h->theta, h->Gtl, h->kk5, h->Vtf, h->rqf, h->resf, s);
    launch_small_accept(NH, k, nevc, h->theta, h->Gtl, h->kk5, h->rqf, h->resf, h->small_acc * sc, tv, 1e-9 * sc,
                        h->lam, h->permf, h->statf, s);
  }
  launch_small_emit(nT, k, h->Vtf, h->permf, h->Vs, s);
  mark(h, PH_PROLONG);
  launch_gemm(false, false, NH, k, NH, 1.0, h->Psi, NH, h->Vs, k, 0.0, h->cc, k, s);   // y_H = L_B^{-T} Phi V
  prolongation_tail(h, k, h->cc);
  h->spec = true;
}

// Retry of a rejected structured solution from a better start block: the k smallest eigenpairs of
// the principal block of Tt on its m lowest coarse modes and the k W-directions (a Rayleigh-Ritz
// approximation of the wanted pairs, Cauchy-interlaced above them), zero-extended to full length.
void structured_retry(pase_handle* h, int k) {
  hipStream_t s = h->stream;
  const int NH = (int)h->lev[h->L].N;
  const int m = std::max(1, std::min(NH, 384 - k));
  const int nr = m + k;
  mark(h, PH_SMALL);
  launch_small_principal(NH, m, k, h->theta, h->Gtl, h->kk5, h->Tm, s);
  syev_any(nr, k, h->Tm, h->rqf, h->Vs, h->syw, h->info + 6, s);
  launch_small_expand(NH, m, k, h->Vs, h->X0f, s);
  launch_fill_int(4, 0, h->statf, s);
  h->retried = true;
  structured_attempt(h, k);
}

// Retry of a structured solution rejected on residuals alone (its order and count were not
// reached): that block, emitted in ascending order into Vs, is close to converged, so the
// Rayleigh-quotient iteration restarts from it, each pair from its own Rayleigh quotient.
void structured_polish(pase_handle* h, int k) {
  hipStream_t s = h->stream;
  const int NH = (int)h->lev[h->L].N;
  mark(h, PH_SMALL);
  launch_copy((size_t)(NH + k) * k, h->Vs, h->X0f, s);
  launch_fill_int(4, 0, h->statf, s);
  h->retried = true;
  structured_attempt(h, k);
}

// ---------------------------------------------------------------- PRECOND-A and GCG_AUG (Sec. 4)
// V_H is level gc.  The fine directions W are replaced by their A-orthogonal complement
// W~ = W - I_H^h a_hat against V_H (a_hat ~ A_H^{-1} I_h^H A W), which is the congruence of eq.
// (Transformation_0) written on vectors: in the basis [I_H^h, W~] the augmented pencil is
//   A~ = [[A_H, a~], [a~^T, alpha~]],  B~ = [[B_H, b~], [b~^T, beta~]],
// a~ = I_h^H A W~ (zero for an exact a_hat, the pencil of eq. Eigen_Problem_Hh_2; here a_hat comes
// from a few CG steps, and the small a~ that remains is kept so that the pencil stays exactly the
// augmented problem), alpha~ = W~^T A W~, b~ = I_h^H M W~, beta~ = W~^T M W~.  GCG_AUG (Alg. 4)
// then works on augmented blocks of gNH + k rows.

constexpr int kAhatSteps = 6;      // CG steps for a_hat (V-cycle from level gc preconditions them)
constexpr int kGcgMaxIter = 50;    // GCG_AUG iterations per correction at most
constexpr int kGcgStall = 4;       // ... and at most this many without a new low of the largest residual
constexpr double kGcgTolFloor = 1e-11;

// composite restriction to level c: xc (N_c x k) = I_h^H xf; and prolongation xf (=, +=, -=) I_H^h xc
void restrict_to(pase_handle* h, int c, int k, const double* xf, double* xc) {
  const double* src = xf;
  for (int l = 0; l < c; ++l) {
    double* dst = (l + 1 == c) ? xc : h->vr[l + 1];
    xfer_restrict(h, l, k, src, dst, 0);
    src = dst;
  }
}

void prolong_from(pase_handle* h, int c, int k, const double* xc, double* xf, int mode) {
  const double* src = xc;
  for (int l = c; l >= 1; --l) {
    double* dst = (l == 1) ? xf : h->vxa[l - 1];
    xfer_prolong(h, l, k, src, dst, (l == 1) ? mode : 0, 0);
    src = dst;
  }
}

// AY = A~ Y and BY = B~ Y for an augmented block Y of w columns (kb fine directions; either output
// may be null): the coarse stencils on the first gNH rows, the couplings as tall-skinny products.
void aug_apply(pase_handle* h, int kb, int w, const double* Y, double* AY, double* BY) {
  hipStream_t s = h->stream;
  const long long NH = h->gNH;
  const int nh = (int)NH;
  stencil_op(h, h->gc, w, EPI_AM, Y, nullptr, AY, BY);
  const double* Yg = Y + NH * w;
  const double* cpl[2] = {h->g_at, h->g_bt};
  const double* blk[2] = {h->g_alt, h->g_bet};
  double* out[2] = {AY, BY};
  for (int o = 0; o < 2; ++o) {
    if (!out[o]) continue;
    launch_gemm(false, false, nh, w, kb, 1.0, cpl[o], kb, Yg, w, 1.0, out[o], w, s);       // += c y_g
    launch_gram_tn(NH, kb, w, cpl[o], kb, Y, w, h->gpart, out[o] + NH * w, s);           // c^T y_H
    launch_gemm(false, false, kb, w, kb, 1.0, blk[o], kb, Yg, w, 1.0, out[o] + NH * w, w, s);
  }
}

// Z = diag(V-cycle on A_H from level gc, alpha~^{-1}) R
void aug_precond(pase_handle* h, int kb, int w, const double* R, double* Z) {
  const long long NH = h->gNH;
  vcycle(h, h->gc, w, R, Z);
  launch_gemm(false, false, kb, w, kb, 1.0, h->g_alinv, kb, R + NH * w, w, 0.0, Z + NH * w, w, h->stream);
}

// Step 2 of Alg. 4: s CG steps per column on A~ x = F from X0, preconditioned by aug_precond
void aug_pcg(pase_handle* h, int kb, int w, const double* F, const double* X0, double* X) {
  hipStream_t s = h->stream;
  const long long Na = h->gNH + kb;
  double *R = h->gR, *Z = h->gZ, *P = h->gPp, *Q = h->gQ;
  aug_apply(h, kb, w, X0, Q, nullptr);
  launch_sub(Na * w, F, Q, R, s);
  aug_precond(h, kb, w, R, Z);
  coldot(h, Na, w, R, Z, h->rho);
  std::swap(Z, P);
  launch_copy((size_t)Na * w, X0, X, s);
  for (int j = 0; j < h->opt.cg_steps; ++j) {
    aug_apply(h, kb, w, P, Q, nullptr);
    coldot(h, Na, w, P, Q, h->pq);
    launch_pcg_alpha(w, h->rho, h->pq, h->alpha, s);
    launch_axpy2(Na, w, h->alpha, P, Q, X, R, s);
    if (j + 1 < h->opt.cg_steps) {
      aug_precond(h, kb, w, R, Z);
      coldot(h, Na, w, R, Z, h->rho2);
      launch_pcg_beta(w, h->rho2, h->rho, h->beta, s);
      launch_xpby(Na, w, Z, h->beta, P, s);
      std::swap(h->rho, h->rho2);
    }
  }
}

// a_hat = A_H^{-1} a approximately: kAhatSteps CG steps from zero on level gc (g_a -> g_ahat)
void ahat_solve(pase_handle* h, int kb) {
  hipStream_t s = h->stream;
  const long long NH = h->gNH;
  const int c = h->gc;
  double *R = h->gR, *Z = h->gZ, *P = h->gPp, *Q = h->gQ, *X = h->g_ahat;
  launch_copy((size_t)NH * kb, h->g_a, R, s);
  launch_sub(NH * kb, nullptr, nullptr, X, s);
  vcycle(h, c, kb, R, Z);
  coldot(h, NH, kb, R, Z, h->rho);
  std::swap(Z, P);
  for (int j = 0; j < kAhatSteps; ++j) {
    stencil_op(h, c, kb, EPI_AM, P, nullptr, Q, nullptr);
    coldot(h, NH, kb, P, Q, h->pq);
    launch_pcg_alpha(kb, h->rho, h->pq, h->alpha, s);
    launch_axpy2(NH, kb, h->alpha, P, Q, X, R, s);
    if (j + 1 < kAhatSteps) {
      vcycle(h, c, kb, R, Z);
      coldot(h, NH, kb, R, Z, h->rho2);
      launch_pcg_beta(kb, h->rho2, h->rho, h->beta, s);
      launch_xpby(NH, kb, Z, h->beta, P, s);
      std::swap(h->rho, h->rho2);
    }
  }
}

// Steps 4-5 of Alg. 3 on the GCG_AUG path, from W in h->X: the complement W~ (in place), the
// couplings and Grams, and alpha~^{-1} for the preconditioner.
void gcg_projection(pase_handle* h, int k) {
  hipStream_t s = h->stream;
  const long long N = h->lev[0].N;
  const int c = h->gc;
  double* W = h->X;
  apply_AM(h, 0, k, W, h->W2, nullptr);
  restrict_to(h, c, k, h->W2, h->g_a);                    // a = I_h^H A W
  ahat_solve(h, k);
  prolong_from(h, c, k, h->g_ahat, W, 2);                 // W~ = W - I_H^h a_hat
  apply_AM(h, 0, k, W, h->W2, h->W3);                     // A W~, M W~
  restrict_to(h, c, k, h->W2, h->g_at);                   // a~
  restrict_to(h, c, k, h->W3, h->g_bt);                   // b~
  launch_gram2_sym(N, k, W, h->W2, h->W3, h->partial, gram_tiles(N, k), h->g_alt, h->g_bet, s);
  launch_symmetrize(k, h->g_alt, s);
  launch_symmetrize(k, h->g_bet, s);
  launch_copy((size_t)k * k, h->g_alt, h->kk2, s);
  launch_cholinv(k, h->kk2, h->info + 1, s);               // alpha~ = L L^T, kk2 <- L^{-1}
  launch_ltl(k, h->kk2, h->g_alinv, s);                    // alpha~^{-1} = L^{-T} L^{-1}
}

// X <- X C, AX <- AX C, BX <- BX C (w x w), through the spare buffers
void gcg_rotate(pase_handle* h, long long Na, int w, const double* C) {
  hipStream_t s = h->stream;
  launch_tsmm(Na, w, h->gX, C, h->gXn, 0, 0, s);
  launch_tsmm(Na, w, h->gAX, C, h->gAXn, 0, 0, s);
  launch_tsmm(Na, w, h->gBX, C, h->gBXn, 0, 0, s);
  std::swap(h->gX, h->gXn);
  std::swap(h->gAX, h->gAXn);
  std::swap(h->gBX, h->gBXn);
}

// GCG_AUG (Alg. 4) for the k smallest pairs of (A~, B~) from the start block [a_hat ; I] (the fine
// directions themselves); the Ritz values end in glam and the vectors in gX.  One synchronisation
// per iteration reads the residuals that choose the active pairs.
pase_status gcg_small(pase_handle* h, int k) {
  hipStream_t s = h->stream;
  const long long NH = h->gNH, Na = NH + k;
  launch_fill_int(5, 0, h->info + 11, s);
  // step 1: two Cholesky-QR passes in B~, then the Rayleigh-Ritz of the start block
  launch_aug_start(NH, k, h->g_ahat, h->gX, s);
  for (int pass = 0; pass < 2; ++pass) {
    aug_apply(h, k, k, h->gX, nullptr, h->gBX);
    launch_gram(Na, k, h->gX, h->gBX, h->partial, gram_tiles(Na, k), h->gGxx, s);
    launch_symmetrize(k, h->gGxx, s);
    launch_cholinv(k, h->gGxx, h->info + 11, s);
    launch_tsmm(Na, k, h->gX, h->gGxx, h->gXn, 0, 1, s);
    std::swap(h->gX, h->gXn);
  }
  aug_apply(h, k, k, h->gX, h->gAX, h->gBX);
  launch_gram(Na, k, h->gX, h->gAX, h->partial, gram_tiles(Na, k), h->gGxx, s);
  launch_symmetrize(k, h->gGxx, s);
  syev_any(k, k, h->gGxx, h->glam, h->gC, h->gsyw, h->info + 12, s);
  gcg_rotate(h, Na, k, h->gC);
  std::vector<double> tol(k, kGcgTolFloor);
  if (h->tolv_on && h->opt.aug_rtol > 0.0)
    for (int j = 0; j < k && j < (int)h->outer_res.size(); ++j)
      tol[j] = std::max(kGcgTolFloor, h->opt.aug_rtol * h->outer_res[j]);
  std::vector<int> act;
  int kp = 0, kp_prev = 0, it = 0, since = 0;
  double best = 1e300;
  bool retried = false;
  while (true) {
    launch_aug_resid(Na, k, h->gAX, h->gBX, h->glam, h->gR, s);
    coldot(h, Na, k, h->gR, h->gR, h->gnorm);
    coldot(h, Na, k, h->gBX, h->gBX, h->gnorm + k);
    HIPC(hipGetLastError());
    HIPC(hipMemcpyAsync(h->pin_gnorm, h->gnorm, sizeof(double) * 2 * k, hipMemcpyDeviceToHost, s));
    HIPC(hipMemcpyAsync(h->pin_lam, h->glam, sizeof(double) * k, hipMemcpyDeviceToHost, s));
    HIPC(hipMemcpyAsync(h->pin_info, h->info, sizeof(int) * 16, hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    const int* inf = h->pin_info;
    if (inf[11] || inf[12]) return fail(h, PASE_E_BREAKDOWN, "GCG_AUG: the start block is not B-orthonormalisable");
    if (inf[13] || inf[14] || inf[15]) {
      // the last iteration's orthonormalisation or Rayleigh-Ritz broke down: back to its start
      // block, and once more without the P block; a second breakdown ends the iteration there
      std::swap(h->gX, h->gXn);
      std::swap(h->gAX, h->gAXn);
      std::swap(h->gBX, h->gBXn);
      std::swap(h->glam, h->glamn);
      launch_fill_int(3, 0, h->info + 13, s);
      ++h->aug_restarts;
      if (retried || kp_prev == 0) break;
      retried = true;
      kp = 0;
      continue;
    }
    double worst = 0.0;
    act.clear();
    for (int j = 0; j < k; ++j) {
      const double res = std::sqrt(h->pin_gnorm[j]) / (std::fabs(h->pin_lam[j]) * std::sqrt(h->pin_gnorm[k + j]));
      if (!std::isfinite(res)) return fail(h, PASE_E_BREAKDOWN, "GCG_AUG: non-finite residual");
      if (res > tol[j]) {
        act.push_back(j);
        worst = std::max(worst, res);
      }
    }
    if (!act.empty()) {
      if (worst < best) {
        best = worst;
        since = 0;
      } else {
        ++since;
      }
    }
    if (act.empty() || it >= kGcgMaxIter || since >= kGcgStall) break;
    const int ka = (int)act.size();
    std::memcpy(h->pin_idx, act.data(), sizeof(int) * ka);
    HIPC(hipMemcpyAsync(h->gidx, h->pin_idx, sizeof(int) * ka, hipMemcpyHostToDevice, s));
    // step 2: W = A~^{-1} (B~ X Lambda) approximately, from X, for the active pairs (shift 0)
    launch_gather_scale(Na, k, ka, h->gidx, h->gBX, h->glam, h->gAW, s);    // F
    launch_gather_scale(Na, k, ka, h->gidx, h->gX, nullptr, h->gBW, s);     // X0
    aug_pcg(h, k, ka, h->gAW, h->gBW, h->gW);
    aug_apply(h, k, ka, h->gW, nullptr, h->gBW);
    // step 3: Y = [P, W] made B~-orthogonal to X and B~-orthonormal, two passes.  The images of
    // Y are applied afresh after each change of Y: the remainders of nearly converged pairs are
    // small, and carrying A~ Y, B~ Y through the scaling of Cholesky-QR would scale their
    // rounding errors up with them.
    const int ny = kp + ka;
    if (kp) launch_copy_cols(Na, kp, ny, kp, h->gP, h->gY, 0, s);
    launch_copy_cols(Na, ka, ny, ka, h->gW, h->gY + kp, 0, s);
    if (kp) launch_copy_cols(Na, kp, ny, kp, h->gBP, h->gBY, 0, s);
    launch_copy_cols(Na, ka, ny, ka, h->gBW, h->gBY + kp, 0, s);
    launch_fill_int(3, 0, h->info + 13, s);
    for (int pass = 0; pass < 2; ++pass) {
      launch_gram_tn(Na, k, ny, h->gX, k, h->gBY, ny, h->gpart, h->gS, s);           // S = X^T B~ Y
      launch_gemm(false, false, (int)Na, ny, k, -1.0, h->gX, k, h->gS, ny, 1.0, h->gY, ny, s);
      aug_apply(h, k, ny, h->gY, nullptr, h->gBY);
      launch_gram_tn(Na, ny, ny, h->gY, ny, h->gBY, ny, h->gpart, h->gG, s);         // Y^T B~ Y
      launch_symmetrize(ny, h->gG, s);
      // factor the unit-diagonal D G D (the remainders' norms span many orders, and the
      // Cholesky's breakdown test is relative to the largest diagonal entry): Li = L^{-1} D
      launch_unit_diag(ny, h->gG, h->gnorm, s);
      launch_cholesky_large(ny, h->gG, ny, h->gchs, h->info + 13 + pass, s);
      launch_trinv_large(ny, h->gG, ny, h->gLi, ny, h->gchs, s);
      launch_scale_cols_sq(ny, h->gLi, h->gnorm, s);
      launch_gemm(false, true, (int)Na, ny, ny, 1.0, h->gY, ny, h->gLi, ny, 0.0, h->gY2, ny, s);
      std::swap(h->gY, h->gY2);
      aug_apply(h, k, ny, h->gY, pass == 1 ? h->gAY : nullptr, h->gBY);
    }
    // step 4: Rayleigh-Ritz on [X, Y]
    const int n = k + ny;
    launch_gram(Na, k, h->gX, h->gAX, h->partial, gram_tiles(Na, k), h->gGxx, s);
    launch_gram_tn(Na, k, ny, h->gX, k, h->gAY, ny, h->gpart, h->gGxy, s);
    launch_gram_tn(Na, ny, ny, h->gY, ny, h->gAY, ny, h->gpart, h->gGyy, s);
    launch_assemble_rr(k, ny, h->gGxx, h->gGxy, h->gGyy, h->gH, s);
    syev_any(n, k, h->gH, h->glamn, h->gC, h->gsyw, h->info + 15, s);
    // X_new = X C_X + Y C_Y (and its images), into the spare buffers
    const double* Cy = h->gC + (size_t)k * k;
    const double* xs[3] = {h->gX, h->gAX, h->gBX};
    const double* ys[3] = {h->gY, h->gAY, h->gBY};
    double* xn[3] = {h->gXn, h->gAXn, h->gBXn};
    for (int q = 0; q < 3; ++q) {
      launch_gemm(false, false, (int)Na, k, k, 1.0, xs[q], k, h->gC, k, 0.0, xn[q], k, s);
      launch_gemm(false, false, (int)Na, k, ny, 1.0, ys[q], ny, Cy, k, 1.0, xn[q], k, s);
    }
    // step 6: P = Y C_Y for the active pairs (the part of X_new outside X)
    launch_gather_cols(ny, k, ka, h->gidx, Cy, h->gCJ, s);
    double* pn[3] = {h->gPn, nullptr, h->gBPn};   // A~ P is not needed: A~ Y is applied afresh
    for (int q = 0; q < 3; q += 2)
      launch_gemm(false, false, (int)Na, ka, ny, 1.0, ys[q], ny, h->gCJ, ka, 0.0, pn[q], ka, s);
    std::swap(h->gX, h->gXn);
    std::swap(h->gAX, h->gAXn);
    std::swap(h->gBX, h->gBXn);
    std::swap(h->gP, h->gPn);
    std::swap(h->gBP, h->gBPn);
    std::swap(h->glam, h->glamn);
    kp_prev = kp;
    kp = ka;
    ++it;
  }
  h->aug_iters += it;
  return PASE_OK;
}

// One correction from (lam, U), U^T M U = I, with R = lam M U - A U already in h->R: everything
// up to the new U in h->U is enqueued; with the structured small solver the result is speculative
// (h->spec) until correction_resolve has seen its status.
pase_status correction_enqueue(pase_handle* h, int k) {
  hipStream_t s = h->stream;
  const long long N = h->lev[0].N;
  const int NH = (int)h->lev[h->L].N;
  // (a) fine solves A w = lam M u from w = u: s CG steps per column
  mark(h, PH_FINE);
  const int ka = (h->ka > 0 && h->ka < k) ? h->ka : k;
  h->fine_cols += ka;
  if (ka < k) {
    // soft locking: the active columns of U and R gathered into W2, W3 (leading dimension ka), their
    // fine solves into R (free until the next residual), then W = U with the active columns replaced
    // plain FP64 with two CG steps, and the mixed form: the last update reads U and writes W in one
    // pass over their full rows (the solved columns updated, the locked ones copied): no gathered U
    // and no merge
    const bool direct = (h->opt.precision == PASE_PREC_FP64 && h->opt.cg_steps == 2) ||
                        h->opt.precision == PASE_PREC_MIXED;
    if (!direct) launch_gather_cols(N, k, ka, h->lock_idx, h->U, h->W2, s);
    launch_gather_cols(N, k, ka, h->lock_idx, h->R, h->W3, s);
    if (h->opt.precision == PASE_PREC_MIXED) {
      pcg_correction_f32(h, ka, h->U, h->W3, h->X, h->lock_idx + h->K, k);
    } else if (direct) {
      pcg(h, ka, h->U, h->X, h->W3, h->lock_idx + h->K, k);
    } else if (h->opt.precision == PASE_PREC_LEARNED) {
      if (!h->net) return fail(h, PASE_E_ARG, "the learned form needs a network (pase_attach_unet)");
      int sw = 0;
      const pase_status st = learned_pcg(h, ka, h->W2, h->R, h->W3, &sw, h->X);   // X is free until the copy
      if (st) return st;
      h->fallbacks += sw;
    } else {
      pcg(h, ka, h->W2, h->R, h->W3);
    }
    if (!direct) launch_merge_cols(N, k, ka, h->lock_idx + h->K, h->R, h->U, h->X, s);
  } else if (h->opt.precision == PASE_PREC_MIXED) {
    pcg_correction_f32(h, k, h->U, h->R, h->X);
  } else if (h->opt.precision == PASE_PREC_LEARNED) {
    if (!h->net) return fail(h, PASE_E_ARG, "the learned form needs a network (pase_attach_unet)");
    int sw = 0;
    const pase_status st = learned_pcg(h, k, h->U, h->X, h->R, &sw, h->W2);
    if (st) return st;
    h->fallbacks += sw;
  } else {
    pcg(h, k, h->U, h->X, h->R);
  }
  double* W = h->X;
  mark(h, PH_PROJECTION);
  if (h->gcg) {
    // PRECOND-A and GCG_AUG (Alg. 5): transform, solve, and u = I_H^h u~_H + W~ gamma~
    gcg_projection(h, k);
    mark(h, PH_SMALL);
    h->spec = false;
    const pase_status st = gcg_small(h, k);
    if (st) return st;
    h->last_path = 4;
    mark(h, PH_PROLONG);
    launch_copy((size_t)k, h->glam, h->lam, s);
    prolong_from(h, h->gc, k, h->gX, h->U, 0);
    launch_tsmm(N, k, h->X, h->gX + (size_t)h->gNH * k, h->U, 1, 0, s);
    return PASE_OK;
  }
  // (b) complement W_perp = W - P c, c = B_H^{-1} P^T M W, and the projection: a = P^T A W_perp,
  // alpha = W_perp^T A W_perp, beta = W_perp^T M W_perp
  if (h->proj_lp) {
    // W_perp formed on the fine grid (the low-precision products below take it)
    apply_AM(h, 0, k, W, nullptr, h->W3);
    restrict_all(h, k, h->W3, h->ca);
    launch_gemm(false, false, NH, k, NH, 1.0, h->BHinv, NH, h->ca, k, 0.0, h->cb, k, s);
    prolong_all(h, k, h->cb, W, 2);
    if (h->fast) launch_copy((size_t)NH * k, h->ca, h->cmw, s);   // P^T M W: W's coarse coordinates
    h->w_perp = true;
    // low-precision projection: W in FP32, FP32 stencils, FP32 restriction, split-BF16 Grams with
    // FP32 K-blocks summed in FP64 (the CG's FP32 vectors are free here)
    float* W32 = h->R32;
    float* AW32 = h->Z32;
    float* MW32 = h->P32;
    launch_d2f((size_t)N * k, W, W32, s);
    stencil_op(h, 0, k, EPI_AM, W32, nullptr, AW32, MW32, 1);
    const float* src = AW32;
    for (int l = 0; l < h->L; ++l) {
      xfer_restrict(h, l, k, src, h->vb32[l + 1], 1);
      src = h->vb32[l + 1];
    }
    launch_f2d((size_t)NH * k, h->vb32[h->L], h->ca, s);
    launch_gram_bf16x3(N, k, W32, AW32, MW32, h->partial, gram_tiles(N, k), h->kk1, h->kk2, s);
    ++h->proj_lp_iters;
  } else {
    // W_perp is not formed: its products follow from W's (one pass of A and M over W, no fine
    // subtraction and no second stencil pass).  With r = P^T A W, m = P^T M W, c = B_H^{-1} m:
    //   a = r - A_H c,  alpha = W^T A W - r^T c - c^T a,  beta = W^T M W - c^T m,
    // and the prolongation takes U = W y_W + P (y_H - c y_W)
    apply_AM(h, 0, k, W, h->W2, h->W3);
    restrict_all(h, k, h->W3, h->ca);                                                       // m
    launch_gemm(false, false, NH, k, NH, 1.0, h->BHinv, NH, h->ca, k, 0.0, h->cb, k, s);   // c
    if (h->fast) launch_copy((size_t)NH * k, h->ca, h->cmw, s);   // P^T M W: W's coarse coordinates
    restrict_all(h, k, h->W2, h->cc);                                                       // r
    launch_gram2_sym(N, k, W, h->W2, h->W3, h->partial, gram_tiles(N, k), h->kk1, h->kk2, s);
    launch_gemm(true, false, k, k, NH, -1.0, h->cb, k, h->ca, k, 1.0, h->kk2, k, s);      // beta
    stencil_op(h, h->L, k, EPI_RESID, h->cb, h->cc, h->ca, nullptr);                       // a = r - A_H c
    launch_gemm(true, false, k, k, NH, -1.0, h->cc, k, h->cb, k, 1.0, h->kk1, k, s);
    launch_gemm(true, false, k, k, NH, -1.0, h->cb, k, h->ca, k, 1.0, h->kk1, k, s);      // alpha
    launch_copy((size_t)NH * k, h->cb, h->cperp, s);
    h->w_perp = false;
  }
  launch_symmetrize(k, h->kk1, s);
  launch_symmetrize(k, h->kk2, s);
  if (h->fast) launch_copy((size_t)k * k, h->kk2, h->kkb, s);
  launch_cholinv(k, h->kk2, h->info + 1, s);               // beta = L L^T, kk2 <- L^{-1}
  launch_copy((size_t)k * k, h->kk2, h->kk3, s);           // Li
  // H = Li alpha Li^T
  launch_gemm(false, false, k, k, k, 1.0, h->kk3, k, h->kk1, k, 0.0, h->kk4, k, s);
  launch_gemm(false, true, k, k, k, 1.0, h->kk4, k, h->kk3, k, 0.0, h->kk5, k, s);
  launch_symmetrize(k, h->kk5, s);
  // (c) small problem
  mark(h, PH_SMALL);
  h->last_path = 0;
  h->spec = false;
  if (h->fast && h->try_fast) {
    // structured path in the eigenbasis of C0: Gt = Psi^T a Li^T, shifts = the current Ritz values
    launch_fill_int(4, 0, h->statf, s);
    launch_gemm(true, false, NH, k, NH, 1.0, h->Psi, NH, h->ca, k, 0.0, h->cb, k, s);
    launch_gemm(false, true, NH, k, k, 1.0, h->cb, k, h->kk3, k, 0.0, h->Gtl, k, s);
    // start block: the coordinates of W in the new basis, [Psi^T P^T M W ; L^T] (L^T = L^{-1} beta)
    launch_gemm(true, false, NH, k, NH, 1.0, h->Psi, NH, h->cmw, k, 0.0, h->X0f, k, s);
    launch_gemm(false, false, k, k, k, 1.0, h->kk3, k, h->kkb, k, 0.0, h->X0f + (size_t)NH * k, k, s);
    h->retried = false;
    structured_attempt(h, k);
    return PASE_OK;
  }
  return correction_dense_tail(h, k);
}

// Status of a speculative structured solution (statf copied to pin_st and synchronised by the
// caller): bookkeeping, and the dense path when it was rejected.
pase_status correction_resolve(pase_handle* h, int k) {
  if (!h->spec) return PASE_OK;
  h->spec = false;
  const int* st = h->pin_st;
  if (st[0] >= 1 && st[2] == 0) {
    h->last_path = h->retried ? 3 : st[0];
    ++h->fast_hits;
    return PASE_OK;
  }
  h->last_path = (st[2] != 0) ? -3 : (st[1] == 0 ? -1 : -2);
  if (!h->retried) {
    // speculative again: read with the next synchronisation
    if (h->last_path == -1) structured_polish(h, k);
    else structured_retry(h, k);
    return PASE_OK;
  }
  return correction_dense_tail(h, k);
}

// One correction with its small problem resolved before returning (standalone entry points).
pase_status correction(pase_handle* h, int k) {
  pase_status st = correction_enqueue(h, k);
  if (st) return st;
  while (h->spec) {
    HIPC(hipMemcpyAsync(h->pin_st, h->statf, 4 * sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIPC(hipStreamSynchronize(h->stream));
    st = correction_resolve(h, k);
    if (st) return st;
  }
  return st;
}

// ---------------------------------------------------------------- batch scheme (Alg. 7)
// One correction of a batch block (k columns of U, Lambda in lam, R = M U Lambda - A U) with
// shift theta: (c) s CG steps, the complement and the projection, (d) the nsel composite pairs
// nearest theta, (e) the k with the largest component in span(u_hat) (eq. largest_component),
// prolongated into U with their eigenvalues in lam, ascending.
//
// In the basis [P L_B^{-T}, W_perp L^{-T}] of the dense path (B-orthonormal; beta_perp = L L^T)
// the unmodified directions u_hat = W_perp + P B_H^{-1} P^T M W have the coordinates
// Z = [L_B^{-1} P^T M W ; L^T], so for an eigenvector v of T the B-norm of its projection onto
// span(u_hat) is ||L_Z^{-1} Z^T v||^2 with Z^T Z = L_Z L_Z^T.
void batch_correction(pase_handle* h, int k, double theta) {
  hipStream_t s = h->stream;
  const long long N = h->lev[0].N;
  const int NH = (int)h->lev[h->L].N;
  const int nT = NH + k;
  const int nsel = std::min(2 * k, nT);
  mark(h, PH_FINE);
  h->fine_cols += k;
  if (h->opt.precision == PASE_PREC_MIXED) pcg_correction_f32(h, k, h->U, h->R, h->X);
  else pcg(h, k, h->U, h->X, h->R);
  double* W = h->X;
  mark(h, PH_PROJECTION);
  apply_AM(h, 0, k, W, nullptr, h->W3);
  restrict_all(h, k, h->W3, h->bmw);                                   // P^T M W
  launch_gemm(false, false, NH, k, NH, 1.0, h->BHinv, NH, h->bmw, k, 0.0, h->cb, k, s);
  prolong_all(h, k, h->cb, W, 2);                                      // W_perp
  h->w_perp = true;
  apply_AM(h, 0, k, W, h->W2, nullptr);
  restrict_all(h, k, h->W2, h->ca);                                    // a = P^T A W_perp
  launch_gram2_sym(N, k, W, h->W2, h->W3, h->partial, gram_tiles(N, k), h->kk1, h->kk2, s);   // alpha, beta
  launch_symmetrize(k, h->kk1, s);
  launch_symmetrize(k, h->kk2, s);
  launch_copy((size_t)k * k, h->kk2, h->kk4, s);                       // beta_perp
  launch_cholinv(k, h->kk2, h->info + 1, s);                           // kk2 <- L^{-1}
  launch_copy((size_t)k * k, h->kk2, h->kk3, s);                       // Li
  launch_gemm(false, false, k, k, k, 1.0, h->kk3, k, h->kk4, k, 0.0, h->bZ + (size_t)NH * k, k, s);   // L^T
  launch_gemm(false, false, NH, k, NH, 1.0, h->LBinv, NH, h->bmw, k, 0.0, h->bZ, k, s);
  launch_gemm(false, false, k, k, k, 1.0, h->kk3, k, h->kk1, k, 0.0, h->kk4, k, s);
  launch_gemm(false, true, k, k, k, 1.0, h->kk4, k, h->kk3, k, 0.0, h->kk5, k, s);             // H
  launch_symmetrize(k, h->kk5, s);
  // (d) T = [[C0, G], [G^T, H]], G = L_B^{-1} a Li^T; its nsel pairs nearest theta
  mark(h, PH_SMALL);
  launch_gemm(false, false, NH, k, NH, 1.0, h->LBinv, NH, h->ca, k, 0.0, h->cb, k, s);
  launch_gemm(false, true, NH, k, k, 1.0, h->cb, k, h->kk3, k, 0.0, h->cc, k, s);
  launch_set_diag_block(nT, NH, k, h->C0, h->cc, h->kk5, h->Tm, s);
  launch_syev_window(nT, nsel, theta, h->Tm, h->blw, h->bVw, h->bsyw, h->info + 2, s);
  // (e) the selection
  launch_gemm(true, false, k, k, nT, 1.0, h->bZ, k, h->bZ, k, 0.0, h->bGZ, k, s);
  launch_symmetrize(k, h->bGZ, s);
  launch_cholinv(k, h->bGZ, h->info + 5, s);
  launch_gemm(true, false, k, nsel, nT, 1.0, h->bZ, k, h->bVw, nsel, 0.0, h->bS, nsel, s);
  launch_gemm(false, false, k, nsel, k, 1.0, h->bGZ, k, h->bS, nsel, 0.0, h->bY, nsel, s);
  launch_batch_select(k, nsel, h->bY, h->bsel, h->info + 7, s);
  launch_gather_cols(nT, nsel, k, h->bsel, h->bVw, h->Vs, s);
  launch_gather_cols(1, nsel, k, h->bsel, h->blw, h->lam, s);
  mark(h, PH_PROLONG);
  launch_gemm(true, false, NH, k, NH, 1.0, h->LBinv, NH, h->Vs, k, 0.0, h->cb, k, s);          // y_H
  prolongation_tail(h, k, h->cb);
}

struct BatchOut {
  int iters = 0;
  int nconv = 0;
  float ms = 0.f;
};

// Alg. 7 step 3 for the pairs first .. first + nb - 1 with up to g guard pairs on each side:
// the block holds the pairs b0 .. b0 + k - 1 (b0 = first - lo, lo = min(g, first), k = lo + nb + g).
// The batch's pairs (positions lo .. lo + nb - 1 of the block, ascending) go to lam_out and to the
// nb columns of Uout (row stride ldu); res_out (host, optional) gets their residuals.
pase_status batch_run(pase_handle* h, int first, int nb, double tol, double* lam_out, double* Uout, int ldu,
                      double* res_out, BatchOut* bo) {
  hipStream_t s = h->stream;
  const long long N = h->lev[0].N;
  const int NH = (int)h->lev[h->L].N;
  const int g = h->opt.guard;
  const int lo = std::min(g, first);
  const int b0 = first - lo;
  const int k = lo + nb + g;
  if (k > h->K) return fail(h, PASE_E_ARG, "the batch and its guard pairs exceed nev_max + guard");
  if (b0 + k > NH) return fail(h, PASE_E_ARG, "the batch and its guard pairs exceed the coarse space");
  HIPC(hipEventRecord(h->ev0, s));
  h->nmark = 0;
  mark(h, PH_START);
  launch_fill_int(16, 0, h->info, s);
  // (a) the coarse eigenvectors b0 .. b0 + k - 1 interpolated, Lambda = their eigenvalues;
  // (b) theta = the midpoint of the block's first and last coarse eigenvalue
  launch_copy_cols(NH, NH, k, k, h->Psi + b0, h->cb, 0, s);
  prolong_all(h, k, h->cb, h->U, 0);
  launch_copy((size_t)k, h->theta + b0, h->lam, s);
  double th[2];
  HIPC(hipMemcpyAsync(&th[0], h->theta + b0, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPC(hipMemcpyAsync(&th[1], h->theta + b0 + k - 1, sizeof(double), hipMemcpyDeviceToHost, s));
  mark(h, PH_RESIDUAL);
  eig_residual(h, k, h->U, h->R);
  HIPC(hipStreamSynchronize(s));
  const double theta = 0.5 * (th[0] + th[1]);
  std::vector<double> hs(3 * k), hl(k), res(k);
  int it = 0, nconv = 0;
  bool conv = false;
  pase_status result = PASE_OK;
  while (true) {
    batch_correction(h, k, theta);
    ++it;
    // (g) on the pairs of step (e); their residual also starts the post-smoothing
    mark(h, PH_RESIDUAL);
    eig_residual(h, k, h->U, h->R);
    mark(h, -1);
    HIPC(hipGetLastError());
    HIPC(hipMemcpyAsync(h->pin_sums, h->sums, sizeof(double) * 3 * k, hipMemcpyDeviceToHost, s));
    HIPC(hipMemcpyAsync(h->pin_lam, h->lam, sizeof(double) * k, hipMemcpyDeviceToHost, s));
    HIPC(hipMemcpyAsync(h->pin_info, h->info, sizeof(int) * 16, hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    settle_marks(h);
    std::memcpy(hs.data(), h->pin_sums, sizeof(double) * 3 * k);
    std::memcpy(hl.data(), h->pin_lam, sizeof(double) * k);
    const int* inf = h->pin_info;
    if (inf[1] || inf[2] || inf[5] || inf[7]) {
      result = fail(h, PASE_E_BREAKDOWN, "Cholesky of a Gram matrix, the windowed eigensolver or the selection failed");
      break;
    }
    nconv = 0;
    bool finite = true;
    for (int j = 0; j < k; ++j) {
      res[j] = std::sqrt(hs[j]) / (std::fabs(hl[j]) * std::sqrt(hs[k + j]));
      if (!std::isfinite(res[j])) finite = false;
      if (j >= lo && j < lo + nb && res[j] <= tol) ++nconv;
    }
    if (!finite) {
      result = fail(h, PASE_E_BREAKDOWN, "non-finite residual or Ritz value");
      break;
    }
    if (nconv == nb) { conv = true; break; }
    if (it >= h->opt.max_outer) break;
    // (f) post-smoothing from u_hat, then the next (c)'s start residual
    mark(h, PH_FINE);
    h->fine_cols += k;
    if (h->opt.precision == PASE_PREC_MIXED) pcg_correction_f32(h, k, h->U, h->R, h->X);
    else pcg(h, k, h->U, h->X, h->R);
    std::swap(h->U, h->X);
    mark(h, PH_RESIDUAL);
    eig_residual(h, k, h->U, h->R);
  }
  launch_copy_cols(N, k, ldu, nb, h->U + lo, Uout, 0, s);
  HIPC(hipEventRecord(h->ev1, s));
  HIPC(hipMemcpyAsync(lam_out, h->lam + lo, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
  HIPC(hipStreamSynchronize(s));
  settle_marks(h);
  HIPC(hipEventElapsedTime(&bo->ms, h->ev0, h->ev1));
  bo->iters = it;
  bo->nconv = nconv;
  if (res_out) std::memcpy(res_out, res.data() + lo, sizeof(double) * nb);
  if (result != PASE_OK) return result;
  if (!conv) return fail(h, PASE_E_NOTCONV, "max_outer reached before every pair of the batch met tol");
  return PASE_OK;
}

pase_status batch_check(pase_handle* h, double tol, const double* lam_out, const double* U) {
  if (!h) return fail(nullptr, PASE_E_ARG, "null handle");
  if (!h->bsel || !h->Psi || !h->theta)
    return fail(h, PASE_E_UNSUPPORTED,
                "the batch scheme needs the dense small path with the coarsest level's eigenbasis "
                "(small_solver 0, N_H + nev_max + guard <= 3840, nev_max + guard <= 128)");
  if (h->opt.precision == PASE_PREC_LEARNED) return fail(h, PASE_E_UNSUPPORTED, "the batch scheme runs in fp64 or mixed");
  if (!lam_out || !U) return fail(h, PASE_E_ARG, "null argument");
  if (!(tol > 0.0)) return fail(h, PASE_E_ARG, "tol must be positive");
  return PASE_OK;
}

void batch_begin(pase_handle* h, pase_report* rep) {
  h->timing = (rep != nullptr);
  for (double& t : h->t_phase) t = 0.0;
  h->fine_cols = 0;
  h->ka = 0;
  h->spec = false;
  h->proj_lp = false;
}

void batch_report(pase_handle* h, pase_report* rep, int iters, int nconv, double ms) {
  h->timing = false;
  if (!rep) return;
  for (int p = 0; p < PASE_PHASES; ++p) rep->t_phase_ms[p] = h->t_phase[p];
  rep->outer_iters = iters;
  rep->n_converged = nconv;
  rep->ritz_history_rows = 0;
  rep->t_solve_ms = ms;
  rep->small_fast_iters = 0;
  rep->learned_fallbacks = 0;
  rep->lowprec_projection_iters = 0;
  rep->fine_solve_columns = h->fine_cols;
  rep->aug_iters = 0;
  rep->aug_restarts = 0;
}

pase_status read_info(pase_handle* h, int* out, int n) {
  HIPC(hipMemcpyAsync(out, h->info, sizeof(int) * n, hipMemcpyDeviceToHost, h->stream));
  HIPC(hipStreamSynchronize(h->stream));
  return PASE_OK;
}

pase_status check_k(pase_handle* h, int k) {
  if (!h) return fail(nullptr, PASE_E_ARG, "null handle");
  if (k < 1 || k > h->K) return fail(h, PASE_E_ARG, "k must be in [1, nev_max]");
  return PASE_OK;
}

}  // namespace

// ================================================================= C ABI
extern "C" {

void pase_options_default(pase_options* opt) {
  if (!opt) return;
  opt->precision = PASE_PREC_FP64;
  opt->nev_max = 16;
  opt->cg_steps = 2;
  opt->max_outer = 500;
  opt->nu = 2;
  opt->omega = 2.0 / 3.0;
  opt->small_solver = 0;
  opt->locking = 1;
  opt->guard = 0;
  opt->start = 0;
  opt->fallback_ratio = 0.5;
  opt->coarse_level = 0;
  opt->aug_rtol = 1e-2;
}

const char* pase_status_string(pase_status s) {
  switch (s) {
    case PASE_OK: return "ok";
    case PASE_E_ARG: return "invalid argument";
    case PASE_E_HIP: return "HIP runtime error";
    case PASE_E_NOMEM: return "workspace too small";
    case PASE_E_NOTCONV: return "not converged";
    case PASE_E_BREAKDOWN: return "breakdown (non-SPD Gram or non-finite values)";
    case PASE_E_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* pase_last_error(const pase_handle* h) { return h ? h->err.c_str() : g_last_error.c_str(); }

pase_status pase_workspace_bytes(const pase_problem* prob, const pase_options* opt, size_t* bytes) {
  pase_handle* h = nullptr;
  if (!bytes) return fail(h, PASE_E_ARG, "bytes is null");
  const pase_status st = check_problem(prob, opt);
  if (st != PASE_OK) return fail(h, st, "invalid or unsupported problem/options");
  pase_handle tmp;
  tmp.opt = *opt;
  set_levels(&tmp, prob);
  tmp.K = opt->nev_max + opt->guard;
  tmp.fine_general = (prob->tensor != nullptr && !prob->csr);
  *bytes = layout(&tmp, nullptr);
  return PASE_OK;
}

pase_status pase_setup(const pase_problem* prob, const pase_options* opt, void* workspace, size_t workspace_bytes,
                       void* stream, pase_handle** out) {
  pase_handle* h = nullptr;
  if (!out) return fail(h, PASE_E_ARG, "out is null");
  *out = nullptr;
  const pase_status st = check_problem(prob, opt);
  if (st != PASE_OK) return fail(h, st, "invalid or unsupported problem/options");
  if (!workspace) return fail(h, PASE_E_ARG, "workspace is null");
  if (((uintptr_t)workspace) & 255) return fail(h, PASE_E_ARG, "workspace must be 256-byte aligned");
  h = new pase_handle();
  h->prob = *prob;
  h->opt = *opt;
  h->stream = (hipStream_t)stream;
  set_levels(h, prob);
  h->K = opt->nev_max + opt->guard;
  h->fine_general = (prob->tensor != nullptr && !prob->csr);
  const size_t need = layout(h, nullptr);
  if (workspace_bytes < need) {
    const pase_status r = fail(h, PASE_E_NOMEM, "workspace smaller than pase_workspace_bytes");
    delete h;
    return r;
  }
  layout(h, workspace);
  h->lev[0].kappa = h->kappa;
  h->kappa_is_one = (prob->kappa == nullptr && !h->fine_general && !h->alg);
  hipStream_t s = h->stream;
  auto bail = [&](pase_status r) {
    g_last_error = h->err;
    if (h->ev0) (void)hipEventDestroy(h->ev0);
    if (h->ev1) (void)hipEventDestroy(h->ev1);
    for (hipEvent_t e : h->evm)
      if (e) (void)hipEventDestroy(e);
    if (h->pin) (void)hipHostFree(h->pin);
    delete h;
    return r;
  };
#define HIPS(call)                                                                            \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess) {                                                                   \
      fail(h, PASE_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_));                 \
      return bail(PASE_E_HIP);                                                                \
    }                                                                                         \
  } while (0)
  const Level& f = h->lev[0];
  const size_t ne = (size_t)f.n * f.n * (h->dim == 3 ? f.n : 1);
  if (h->alg) {
    // algebraic input: Jacobi diagonals of every level from the given A_l
    for (int l = 0; l <= h->L; ++l) launch_csr_diag_inv(csr_mat(h->csr.A[l]), h->lev[l].N, h->lev[l].dinv, s);
  } else if (prob->kappa) {
    HIPS(hipMemcpyAsync(h->kappa, prob->kappa, ne * sizeof(double), hipMemcpyDeviceToDevice, s));
  } else {
    std::vector<double> ones(ne, 1.0);
    HIPS(hipMemcpyAsync(h->kappa, ones.data(), ne * sizeof(double), hipMemcpyHostToDevice, s));
    HIPS(hipStreamSynchronize(s));
  }
  HIPS(hipMemsetAsync(h->zero16, 0, 8 * sizeof(double), s));
  if (h->alg) {
    // nothing to assemble
  } else if (h->fine_general) {
    launch_assemble_general(f.n, prob->tensor, prob->reaction, h->lev[0].coef, h->lev[0].dinv, s);
  } else {
    launch_kappa_dinv(h->dim, f.n, h->kappa, h->lev[0].dinv, s);
  }
  if (h->logk) launch_node_logk(f.n, h->kappa, h->logk, s);
  // Galerkin stencils A_l = P_l^T A_{l-1} P_l from 3^d colour probes
  const int NS = h->NS;
  for (int l = 1; l <= h->L && !h->alg; ++l) {
    const Level& c = h->lev[l];
    const Level& p = h->lev[l - 1];
    double* E = h->setup_scratch;
    double* PE = E + (size_t)c.N * NS;
    double* APE = PE + (size_t)p.N * NS;
    launch_color_probe(h->dim, c.m, E, s);
    launch_prolong(h->dim, p.m, c.m, NS, E, PE, 0, 0, s);
    apply_AM(h, l - 1, NS, PE, APE, nullptr);
    launch_restrict(h->dim, p.m, c.m, NS, APE, E, 0, s);
    launch_extract_galerkin(h->dim, c.m, E, h->lev[l].coef, h->lev[l].dinv, s);
  }
  // coarse dense factorisations
  const Level& cl = h->lev[h->L];
  const int NH = (int)cl.N;
  double* AL = h->dtmp;
  auto coarse_dense = [&](int mass, double* D) {   // A_L (mass = 0) or M_L, dense
    if (h->alg) launch_csr_to_dense(csr_mat(mass ? h->csr.M[h->L] : h->csr.A[h->L]), cl.N, D, s);
    else launch_stencil_to_dense(h->dim, cl.m, mass ? nullptr : cl.coef, cl.h, mass, D, s);
  };
  coarse_dense(0, AL);
  // blocked factorisations above one workgroup's size; their scratch follows the N_H x N_H
  // product area at the start of the setup scratch
  // blocked factorisations (MFMA panel updates) above 64: the one-workgroup kernels take milliseconds
  // already at N_H = 343
  const bool big_coarse = NH > 64;
  double* lscr = h->setup_scratch + (size_t)NH * NH;
  auto cholesky = [&](double* A, int* inf) {
    if (big_coarse) launch_cholesky_large(NH, A, NH, lscr, inf, s);
    else launch_cholesky(NH, A, NH, inf, s);
  };
  auto trinv = [&](const double* L, double* Li) {
    if (big_coarse) launch_trinv_large(NH, L, NH, Li, NH, lscr, s);
    else launch_trinv(NH, L, NH, Li, NH, s);
  };
  cholesky(AL, h->info + 8);                                         // AL <- L_A
  trinv(AL, h->C0);                                                  // C0 <- L_A^{-1} (temp)
  launch_gemm(true, false, NH, NH, NH, 1.0, h->C0, NH, h->C0, NH, 0.0, h->AinvL, NH, s);
  launch_symmetrize(NH, h->AinvL, s);
  if (h->AinvL32) launch_d2f((size_t)NH * NH, h->AinvL, h->AinvL32, s);
  double* BL = h->dtmp;
  coarse_dense(1, BL);
  cholesky(BL, h->info + 9);                                         // BL <- L_B
  trinv(BL, h->LBinv);
  launch_gemm(true, false, NH, NH, NH, 1.0, h->LBinv, NH, h->LBinv, NH, 0.0, h->BHinv, NH, s);
  launch_symmetrize(NH, h->BHinv, s);
  // C0 = LB^{-1} A_H LB^{-T}
  coarse_dense(0, AL);
  double* tmp = h->setup_scratch;
  launch_gemm(false, false, NH, NH, NH, 1.0, h->LBinv, NH, AL, NH, 0.0, tmp, NH, s);
  launch_gemm(false, true, NH, NH, NH, 1.0, tmp, NH, h->LBinv, NH, 0.0, h->C0, NH, s);
  launch_symmetrize(NH, h->C0, s);
  if (h->fast || h->psi_only) {
    // C0 = Phi diag(theta) Phi^T (all N_H pairs, dense solver), Psi = L_B^{-T} Phi
    HIPS(hipMemcpyAsync(h->Tm, h->C0, sizeof(double) * NH * NH, hipMemcpyDeviceToDevice, s));
    double* Phi = h->dtmp;
    syev_any(NH, NH, h->Tm, h->theta, Phi, h->syw, h->info + 10, s);
    launch_gemm(true, false, NH, NH, NH, 1.0, h->LBinv, NH, Phi, NH, 0.0, h->Psi, NH, s);
  }
  HIPS(hipGetLastError());
  int inf[16];
  HIPS(hipMemcpyAsync(inf, h->info, sizeof(inf), hipMemcpyDeviceToHost, s));
  HIPS(hipStreamSynchronize(s));
  if (inf[8] || inf[9]) {
    fail(h, PASE_E_BREAKDOWN, "coarse Cholesky failed");
    return bail(PASE_E_BREAKDOWN);
  }
  if (h->psi_only && inf[10]) h->psi_only = false;   // no coarse start then
  if (h->fast) {
    if (inf[10]) {
      h->fast = false;   // the dense path stays available
    } else {
      std::vector<double> th(NH);
      HIPS(hipMemcpyAsync(th.data(), h->theta, sizeof(double) * NH, hipMemcpyDeviceToHost, s));
      HIPS(hipStreamSynchronize(s));
      double mx = 1.0;
      for (double t : th) mx = std::max(mx, std::fabs(t));
      h->small_scale = mx;
    }
  }
  HIPS(hipEventCreate(&h->ev0));
  HIPS(hipEventCreate(&h->ev1));
  for (hipEvent_t& e : h->evm) HIPS(hipEventCreate(&e));
  {
    const size_t Kp = (size_t)h->K;
    HIPS(hipHostMalloc(&h->pin, sizeof(double) * 7 * Kp + sizeof(int) * (2 * Kp + 20), hipHostMallocDefault));
    double* pd = (double*)h->pin;
    h->pin_sums = pd;
    h->pin_lam = pd + 3 * Kp;
    h->pin_tolv = pd + 4 * Kp;
    h->pin_gnorm = pd + 5 * Kp;
    int* pi = (int*)(pd + 7 * Kp);
    h->pin_info = pi;
    h->pin_st = pi + 16;
    h->pin_idx = pi + 20;
  }
#undef HIPS
  *out = h;
  return PASE_OK;
}

pase_status pase_destroy(pase_handle* h) {
  if (!h) return PASE_OK;
  if (h->ev0) (void)hipEventDestroy(h->ev0);
  if (h->ev1) (void)hipEventDestroy(h->ev1);
  for (hipEvent_t e : h->evm)
    if (e) (void)hipEventDestroy(e);
  if (h->pin) (void)hipHostFree(h->pin);
  delete h;
  return PASE_OK;
}

pase_status pase_level_size(const pase_handle* h, int level, long long* N) {
  if (!h || !N || level < 0 || level > h->L) return PASE_E_ARG;
  *N = h->lev[level].N;
  return PASE_OK;
}

pase_status pase_apply(pase_handle* h, int level, int k, const double* X, double* AX, double* MX) {
  pase_status st = check_k(h, k);
  if (st) return st;
  if (level < 0 || level > h->L || !X) return fail(h, PASE_E_ARG, "bad level or X");
  apply_AM(h, level, k, X, AX, MX);
  HIPC(hipGetLastError());
  HIPC(hipStreamSynchronize(h->stream));
  return PASE_OK;
}

pase_status pase_vcycle(pase_handle* h, int k, const double* B, double* Z) {
  pase_status st = check_k(h, k);
  if (st) return st;
  if (!B || !Z || B == Z) return fail(h, PASE_E_ARG, "B, Z must be distinct non-null buffers");
  vcycle(h, 0, k, B, Z);
  HIPC(hipGetLastError());
  HIPC(hipStreamSynchronize(h->stream));
  return PASE_OK;
}

pase_status pase_pcg(pase_handle* h, int k, const double* lambda_host, const double* U, double* W) {
  pase_status st = check_k(h, k);
  if (st) return st;
  if (!lambda_host || !U || !W) return fail(h, PASE_E_ARG, "null argument");
  const long long N = h->lev[0].N;
  HIPC(hipMemcpyAsync(h->lam, lambda_host, sizeof(double) * k, hipMemcpyHostToDevice, h->stream));
  eig_residual(h, k, U, h->R);
  if (h->opt.precision == PASE_PREC_LEARNED) {
    if (!h->net) return fail(h, PASE_E_ARG, "the learned form needs a network (pase_attach_unet)");
    int sw = 0;
    st = learned_pcg(h, k, U, h->X, h->R, &sw, h->W2);
    if (st) return st;
    h->fallbacks = sw;
  } else {
    pcg(h, k, U, h->X, h->R);
  }
  launch_copy((size_t)N * k, h->X, W, h->stream);
  HIPC(hipGetLastError());
  HIPC(hipStreamSynchronize(h->stream));
  return PASE_OK;
}

pase_status pase_restrict(pase_handle* h, int k, const double* Xf, double* Xc) {
  pase_status st = check_k(h, k);
  if (st) return st;
  if (!Xf || !Xc) return fail(h, PASE_E_ARG, "null argument");
  restrict_all(h, k, Xf, Xc);
  HIPC(hipGetLastError());
  HIPC(hipStreamSynchronize(h->stream));
  return PASE_OK;
}

pase_status pase_prolong(pase_handle* h, int k, const double* Xc, double* Xf) {
  pase_status st = check_k(h, k);
  if (st) return st;
  if (!Xf || !Xc) return fail(h, PASE_E_ARG, "null argument");
  prolong_all(h, k, Xc, Xf, 0);
  HIPC(hipGetLastError());
  HIPC(hipStreamSynchronize(h->stream));
  return PASE_OK;
}

pase_status pase_gram(pase_handle* h, long long N, int k, const double* X, const double* Y, double* G) {
  pase_status st = check_k(h, k);
  if (st) return st;
  if (!X || !Y || !G || N < 1 || N > h->lev[0].N) return fail(h, PASE_E_ARG, "bad Gram arguments");
  launch_gram(N, k, X, Y, h->partial, gram_tiles(N, k), G, h->stream);
  HIPC(hipGetLastError());
  HIPC(hipStreamSynchronize(h->stream));
  return PASE_OK;
}

pase_status pase_gram_bf16x3(pase_handle* h, long long N, int k, const float* X, const float* Y, double* G) {
  pase_status st = check_k(h, k);
  if (st) return st;
  if (k > 128) return fail(h, PASE_E_ARG, "the split-BF16 Gram needs k <= 128");
  if (!X || !Y || !G || N < 1 || N > h->lev[0].N) return fail(h, PASE_E_ARG, "bad Gram arguments");
  launch_gram_bf16x3(N, k, X, Y, nullptr, h->partial, gram_tiles(N, k), G, nullptr, h->stream);
  HIPC(hipGetLastError());
  HIPC(hipStreamSynchronize(h->stream));
  return PASE_OK;
}

int pase_small_eig_max_n(const pase_handle* h) {
  // a GCG_AUG handle keeps no dense augmented matrix (its Tm, if any, holds the coarse start's C0)
  return (h && h->Tm && !h->gcg) ? std::min(h->nT, syev_large_max_n()) : 0;
}

pase_status pase_small_eig(pase_handle* h, int n, int k, const double* T, double* w_host, double* V) {
  pase_status st = check_k(h, k);
  if (st) return st;
  if (!h->Tm) return fail(h, PASE_E_UNSUPPORTED, "small problem larger than the dense eigensolver supports");
  if (!T || !w_host || !V || n < 2 || n > pase_small_eig_max_n(h) || k > n || k > syev_max_k())
    return fail(h, PASE_E_ARG, "bad small_eig arguments");
  HIPC(hipMemcpyAsync(h->Tm, T, sizeof(double) * n * n, hipMemcpyDeviceToDevice, h->stream));
  syev_any(n, k, h->Tm, h->lam, V, h->syw, h->info + 2, h->stream);
  HIPC(hipGetLastError());
  HIPC(hipMemcpyAsync(w_host, h->lam, sizeof(double) * k, hipMemcpyDeviceToHost, h->stream));
  int inf[16];
  st = read_info(h, inf, 16);
  if (st) return st;
  if (inf[2]) return fail(h, PASE_E_BREAKDOWN, "small eigensolver breakdown");
  return PASE_OK;
}

pase_status pase_correction(pase_handle* h, int k, double* lambda_host, double* U) {
  pase_status st = check_k(h, k);
  if (st) return st;
  if (!h->Tm && !h->gcg)
    return fail(h, PASE_E_UNSUPPORTED, "small problem larger than the dense eigensolver supports");
  if (!lambda_host || !U) return fail(h, PASE_E_ARG, "null argument");
  const long long N = h->lev[0].N;
  hipStream_t s = h->stream;
  HIPC(hipMemsetAsync(h->info, 0, 16 * sizeof(int), s));
  HIPC(hipMemcpyAsync(h->lam, lambda_host, sizeof(double) * k, hipMemcpyHostToDevice, s));
  launch_copy((size_t)N * k, U, h->U, s);
  eig_residual(h, k, h->U, h->R);
  h->ka = 0;
  h->small_acc = 1e-11;
  h->tolv_on = false;
  h->try_fast = true;
  h->proj_lp = false;   // a standalone correction projects in FP64, whatever a solve left behind
  h->nev_cur = k;
  st = correction(h, k);
  if (st) return st;
  launch_copy((size_t)N * k, h->U, U, s);
  HIPC(hipGetLastError());
  HIPC(hipMemcpyAsync(lambda_host, h->lam, sizeof(double) * k, hipMemcpyDeviceToHost, s));
  int inf[16];
  st = read_info(h, inf, 16);
  if (st) return st;
  if (inf[1] || inf[2]) return fail(h, PASE_E_BREAKDOWN, "Gram Cholesky or small eigensolver breakdown");
  return PASE_OK;
}

pase_status pase_solve(pase_handle* h, int nev, double tol, const double* U0, double* lambda_host, double* U,
                       pase_report* rep) {
  pase_status st = check_k(h, nev);
  if (st) return st;
  if (nev > h->opt.nev_max) return fail(h, PASE_E_ARG, "nev must be in [1, nev_max]");
  if (!h->Tm && !h->gcg)
    return fail(h, PASE_E_UNSUPPORTED, "small problem larger than the dense eigensolver supports");
  if (!lambda_host || !U) return fail(h, PASE_E_ARG, "null argument");
  if (h->opt.start == 1 && !((h->fast || h->psi_only) && h->Psi))
    return fail(h, PASE_E_UNSUPPORTED, "the coarse start needs the coarsest level's eigenbasis");
  if (!(tol > 0.0)) return fail(h, PASE_E_ARG, "tol must be positive");
  const int k = nev + h->opt.guard;   // block size: the wanted pairs and the guard pairs
  h->nev_cur = nev;
  const long long N = h->lev[0].N;
  hipStream_t s = h->stream;
  HIPC(hipEventRecord(h->ev0, s));
  h->timing = (rep != nullptr);
  h->nmark = 0;
  for (double& t : h->t_phase) t = 0.0;
  mark(h, PH_START);
  HIPC(hipMemsetAsync(h->info, 0, 16 * sizeof(int), s));
  h->fast_hits = 0;
  h->fallbacks = 0;
  h->proj_lp = (h->opt.precision == PASE_PREC_MIXED && k <= 128 && !h->gcg);   // the split-BF16 Gram's limit
  h->aug_iters = 0;
  h->aug_restarts = 0;
  h->proj_lp_iters = 0;
  h->ka = 0;
  h->fine_cols = 0;
  h->spec = false;
  const bool locking = h->opt.locking != 0;
  double lp_best = 0.0;   // smallest max-residual seen in the first phase
  int lp_stall = 0;       // corrections since it last decreased
  if (h->opt.precision == PASE_PREC_LEARNED && !h->net)
    return fail(h, PASE_E_ARG, "the learned form needs a network (pase_attach_unet)");
  if (h->opt.start == 1) {
    // Alg. 3 steps 1-2: the k smallest eigenvectors of (A_H, B_H) (the first k columns of
    // Psi = L_B^{-T} Phi, B_H-orthonormal), interpolated to the fine mesh
    const int NH = (int)h->lev[h->L].N;
    launch_copy_cols(NH, NH, k, k, h->Psi, h->cb, 0, s);
    prolong_all(h, k, h->cb, h->U, 0);
  } else if (!U0) {
    launch_copy_cols(N, 0, k, 0, nullptr, h->U, 1, s);              // fixed uniform(-1, 1) block
  } else if (k > nev) {
    launch_copy_cols(N, nev, k, nev, U0, h->U, 1, s);               // guard columns: fixed uniform(-1, 1)
  } else {
    launch_copy((size_t)N * k, U0, h->U, s);
  }
  // start: two passes of Cholesky-QR in M, Lambda0 = diag(U^T A U)
  for (int pass = 0; pass < 2; ++pass) cholqr_m(h, k, h->U, h->X, 3 + pass);
  apply_AM(h, 0, k, h->U, h->W2, nullptr);
  coldot(h, N, k, h->U, h->W2, h->lam);
  std::vector<double> hs(3 * k), hl(k);
  int it = 0;
  bool conv = false;
  int nconv = 0;
  std::vector<double> res(k), lit(k);
  int rows = 0;
  pase_status result = PASE_OK;
  while (true) {
    mark(h, PH_RESIDUAL);
    eig_residual(h, k, h->U, h->R);
    mark(h, -1);
    HIPC(hipGetLastError());
    HIPC(hipMemcpyAsync(h->pin_sums, h->sums, sizeof(double) * 3 * k, hipMemcpyDeviceToHost, s));
    HIPC(hipMemcpyAsync(h->pin_lam, h->lam, sizeof(double) * k, hipMemcpyDeviceToHost, s));
    HIPC(hipMemcpyAsync(h->pin_info, h->info, sizeof(int) * 16, hipMemcpyDeviceToHost, s));
    if (h->spec) HIPC(hipMemcpyAsync(h->pin_st, h->statf, 4 * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    settle_marks(h);
    if (h->spec) {
      // the previous correction's structured solution was used speculatively (one synchronisation
      // per correction): on a rejection the dense path redoes the prolongation and the residual
      const bool accepted = h->pin_st[0] >= 1 && h->pin_st[2] == 0;
      st = correction_resolve(h, k);
      if (st) return st;
      if (rep && rep->small_path_host && it - 1 < h->opt.max_outer) rep->small_path_host[it - 1] = h->last_path;
      if (!accepted) continue;
    }
    std::memcpy(hs.data(), h->pin_sums, sizeof(double) * 3 * k);
    std::memcpy(hl.data(), h->pin_lam, sizeof(double) * k);
    const int* inf = h->pin_info;
    if (inf[1] || inf[2] || inf[3] || inf[4])
      return fail(h, PASE_E_BREAKDOWN, "Cholesky of a Gram matrix or the small eigensolver failed");
    nconv = 0;
    bool finite = true;
    for (int j = 0; j < k; ++j) {
      const double rn = std::sqrt(hs[j]);
      res[j] = rn / (std::fabs(hl[j]) * std::sqrt(hs[k + j]));
      lit[j] = rn / (std::fabs(hl[j]) * std::sqrt(hs[2 * k + j]));
      if (!std::isfinite(res[j]) || !std::isfinite(hl[j])) finite = false;
      if (j < nev && res[j] <= tol) ++nconv;   // only the wanted pairs decide convergence
    }
    if (rep && rep->ritz_history_host && rows <= h->opt.max_outer) {
      std::memcpy(rep->ritz_history_host + (size_t)rows * nev, hl.data(), sizeof(double) * nev);
      ++rows;
    }
    if (!finite) {
      result = fail(h, PASE_E_BREAKDOWN, "non-finite residual or Ritz value");
      break;
    }
    if (nconv == nev) { conv = true; break; }
    if (it >= h->opt.max_outer) break;
    {
      // from a start block whose every residual is above 1e-2 (a random one) the Ritz values are
      // too far off for the structured solver's shifts: the first correction goes dense directly
      double mn = 1e300;
      for (int j = 0; j < k; ++j) mn = std::min(mn, res[j]);
      h->try_fast = !(it == 0 && mn > 1e-2 && h->opt.start == 0);
    }
    if (locking) {
      // the next correction's fine solves: wanted pairs with res > tol / 10 and guard pairs with
      // res > 100 tol (they only have to span the space past the wanted ones), ascending order
      h->lock_host.clear();
      int extra = -1;   // an even count keeps the stencils on their two-column vector loads
      for (int j = 0; j < k; ++j) {
        if (!(res[j] <= ((j < nev) ? 0.1 * tol : 100.0 * tol))) h->lock_host.push_back(j);
        else if (extra < 0) extra = j;
      }
      if ((h->lock_host.size() & 1) && extra >= 0)
        h->lock_host.insert(std::lower_bound(h->lock_host.begin(), h->lock_host.end(), extra), extra);
      h->ka = (int)h->lock_host.size();
      if (h->ka > 0 && h->ka < k)
      {
        std::memcpy(h->pin_idx, h->lock_host.data(), sizeof(int) * h->ka);
        int* pos = h->pin_idx + h->K;
        for (int j = 0; j < k; ++j) pos[j] = -1;
        for (int a = 0; a < h->ka; ++a) pos[h->lock_host[a]] = a;
        HIPC(hipMemcpyAsync(h->lock_idx, h->pin_idx, sizeof(int) * (h->K + k), hipMemcpyHostToDevice, s));
      }
    }
    {
      // the augmented problem needs no more accuracy than the outer pairs have: the pair at
      // position j of the ascending order is accepted at residual max(1e-11, 1e-2 res_j) max|theta|
      h->tolv_host.resize(k);
      for (int j = 0; j < k; ++j) h->tolv_host[j] = std::max(1.0, 1e9 * res[j]);   // x 1e-11
      h->outer_res.assign(res.begin(), res.begin() + k);
      h->small_acc = 1e-11;
      h->tolv_on = true;
      std::memcpy(h->pin_tolv, h->tolv_host.data(), sizeof(double) * k);
      HIPC(hipMemcpyAsync(h->small_tolv, h->pin_tolv, sizeof(double) * k, hipMemcpyHostToDevice, s));
    }
    if (h->proj_lp) {
      double mr = 0.0, mn = 1e300;
      for (int j = 0; j < k; ++j) {
        mr = std::max(mr, res[j]);
        mn = std::min(mn, res[j]);
      }
      // phase 2 (FP64 projection) as soon as some pair nears the low-precision projection's
      // accuracy floor (residuals of 1e-6 to 5e-6: a pair below 1e-5), or when the largest
      // residual has not reached a new low for 3 corrections
      if (it == 0 || mr < lp_best) {
        lp_best = mr;
        lp_stall = 0;
      } else {
        ++lp_stall;
      }
      if (mn < 1e-5 || lp_stall >= 3) h->proj_lp = false;
    }
    st = correction_enqueue(h, k);
    if (st) return st;
    if (!h->spec && rep && rep->small_path_host && it < h->opt.max_outer) rep->small_path_host[it] = h->last_path;
    ++it;
  }
  h->ka = 0;   // the standalone correction entry points always run every column
  h->try_fast = true;
  h->proj_lp = false;     // project in FP64
  h->small_acc = 1e-11;   // and use the fixed acceptance tolerance
  h->tolv_on = false;
  if (k > nev) launch_copy_cols(N, k, nev, nev, h->U, U, 0, s);   // the wanted pairs
  else launch_copy((size_t)N * k, h->U, U, s);
  HIPC(hipEventRecord(h->ev1, s));
  HIPC(hipMemcpyAsync(lambda_host, h->lam, sizeof(double) * nev, hipMemcpyDeviceToHost, s));
  HIPC(hipStreamSynchronize(s));
  float ms = 0.f;
  HIPC(hipEventElapsedTime(&ms, h->ev0, h->ev1));
  settle_marks(h);
  h->timing = false;
  if (rep) {
    for (int p = 0; p < PASE_PHASES; ++p) rep->t_phase_ms[p] = h->t_phase[p];
    rep->outer_iters = it;
    rep->n_converged = nconv;
    rep->ritz_history_rows = rows;
    rep->t_solve_ms = ms;
    rep->small_fast_iters = h->fast_hits;
    rep->learned_fallbacks = h->fallbacks;
    rep->lowprec_projection_iters = h->proj_lp_iters;
    rep->fine_solve_columns = h->fine_cols;
    rep->aug_iters = h->aug_iters;
    rep->aug_restarts = h->aug_restarts;
    if (rep->res_host) std::memcpy(rep->res_host, res.data(), sizeof(double) * nev);
    if (rep->res_literal_host) std::memcpy(rep->res_literal_host, lit.data(), sizeof(double) * nev);
  }
  if (result != PASE_OK) return result;
  if (!conv) return fail(h, PASE_E_NOTCONV, "max_outer reached before every pair met tol");
  return PASE_OK;
}

pase_status pase_solve_batch(pase_handle* h, int first, int nb, double tol, double* lambda_host, double* U, int ldu,
                             pase_report* rep) {
  pase_status st = batch_check(h, tol, lambda_host, U);
  if (st) return st;
  if (first < 0 || nb < 1 || ldu < nb) return fail(h, PASE_E_ARG, "need first >= 0, nb >= 1 and ldu >= nb");
  batch_begin(h, rep);
  BatchOut bo;
  st = batch_run(h, first, nb, tol, lambda_host, U, ldu, rep ? rep->res_host : nullptr, &bo);
  batch_report(h, rep, bo.iters, bo.nconv, bo.ms);
  return st;
}

pase_status pase_solve_batches(pase_handle* h, int m, int nb, double tol, double* lambda_host, double* U,
                               pase_report* rep) {
  pase_status st = batch_check(h, tol, lambda_host, U);
  if (st) return st;
  if (m < 1 || nb < 1) return fail(h, PASE_E_ARG, "need m >= 1 and nb >= 1");
  batch_begin(h, rep);
  int iters = 0, nconv = 0;
  double ms = 0.0;
  double t_phase[PASE_PHASES] = {};
  // Alg. 7 step 4: the batches one after another, batch i into columns first .. first + k_i - 1
  for (int first = 0; first < m && st == PASE_OK; first += nb) {
    const int k = std::min(nb, m - first);
    BatchOut bo;
    for (double& t : h->t_phase) t = 0.0;
    double* ro = (rep && rep->res_host) ? rep->res_host + first : nullptr;
    st = batch_run(h, first, k, tol, lambda_host + first, U + first, m, ro, &bo);
    iters += bo.iters;
    nconv += bo.nconv;
    ms += bo.ms;
    for (int p = 0; p < PASE_PHASES; ++p) t_phase[p] += h->t_phase[p];
  }
  for (int p = 0; p < PASE_PHASES; ++p) h->t_phase[p] = t_phase[p];
  batch_report(h, rep, iters, nconv, ms);
  return st;
}

pase_status pase_attach_unet(pase_handle* h, pase_unet* u) {
  if (!h || !u) return fail(h, PASE_E_ARG, "null argument");
  if (h->opt.precision != PASE_PREC_LEARNED) return fail(h, PASE_E_ARG, "the handle is not set up for the learned form");
  if (unet_fine_n(u) != h->lev[0].n) return fail(h, PASE_E_ARG, "the network was created for another fine mesh");
  if (unet_batch_max(u) < h->K) return fail(h, PASE_E_ARG, "the network's batch_max is below nev_max + guard");
  unet_set_stream(u, h->stream);
  h->net = u;
  return PASE_OK;
}

pase_status pase_harvest(pase_handle* h, int k, const double* lambda_host, const double* U, double* R, double* V) {
  pase_status st = check_k(h, k);
  if (st) return st;
  if (!lambda_host || !U || !R || !V || R == V || U == R || U == V)
    return fail(h, PASE_E_ARG, "U, R, V must be distinct non-null buffers");
  hipStream_t s = h->stream;
  HIPC(hipMemcpyAsync(h->lam, lambda_host, sizeof(double) * k, hipMemcpyHostToDevice, s));
  eig_residual(h, k, U, R);
  vcycle(h, 0, k, R, V);
  HIPC(hipGetLastError());
  HIPC(hipStreamSynchronize(s));
  return PASE_OK;
}

pase_status pase_fine_diag_inverse(pase_handle* h, double* dinv) {
  if (!h || !dinv) return fail(h, PASE_E_ARG, "null argument");
  HIPC(hipMemcpyAsync(dinv, h->lev[0].dinv, sizeof(double) * h->lev[0].N, hipMemcpyDeviceToDevice, h->stream));
  HIPC(hipStreamSynchronize(h->stream));
  return PASE_OK;
}

pase_status pase_export_csr(pase_handle* h, int level, int which, int* rows, int* cols, int* slots, int* rowptr,
                            int* colind, double* val) {
  if (!h || !rows || !cols || !slots) return fail(h, PASE_E_ARG, "null argument");
  if (h->alg) return fail(h, PASE_E_UNSUPPORTED, "the handle's operators are already CSR matrices");
  if (level < 0 || level > h->L || which < 0 || which > 3 || (which >= 2 && level < 1))
    return fail(h, PASE_E_ARG, "level or which out of range");
  const int dim = h->dim;
  const int ns = dim == 3 ? 27 : 9;
  const Level& lv = h->lev[level];
  if (which <= 1) {
    *rows = *cols = (int)lv.N;
    *slots = ns;
  } else if (which == 2) {
    *rows = (int)h->lev[level - 1].N;
    *cols = (int)lv.N;
    *slots = 1 << dim;
  } else {
    *rows = (int)lv.N;
    *cols = (int)h->lev[level - 1].N;
    *slots = ns;
  }
  if (!rowptr && !colind && !val) return PASE_OK;
  if (!rowptr || !colind || !val) return fail(h, PASE_E_ARG, "rowptr, colind and val go together");
  if ((long long)*rows * *slots > 0x7fffffffLL) return fail(h, PASE_E_UNSUPPORTED, "more than 2^31 entries");
  hipStream_t s = h->stream;
  if (which == 0) {
    // the level's A stencil; the fine level's comes from kappa (coefficients formed into the
    // setup scratch) unless it is assembled already
    const double* coef = lv.coef;
    if (level == 0 && !h->fine_general) {
      // the setup scratch (the fine multi-vectors' space, free between solves) holds at least
      // 3 N_0 3^dim doubles
      double* tmp = h->setup_scratch;
      launch_kappa_coefs(dim, lv.n, h->kappa_is_one ? nullptr : h->kappa, tmp, s);
      coef = tmp;
    }
    launch_export_stencil(dim, lv.m, coef, lv.h, rowptr, colind, val, s);
  } else if (which == 1) {
    launch_export_stencil(dim, lv.m, nullptr, lv.h, rowptr, colind, val, s);
  } else if (which == 2) {
    launch_export_prolong(dim, h->lev[level - 1].m, lv.m, rowptr, colind, val, s);
  } else {
    launch_export_restrict(dim, h->lev[level - 1].m, lv.m, rowptr, colind, val, s);
  }
  HIPC(hipGetLastError());
  HIPC(hipStreamSynchronize(s));
  return PASE_OK;
}

pase_status pase_node_logk(pase_handle* h, double* logk) {
  if (!h || !logk) return fail(h, PASE_E_ARG, "null argument");
  if (h->dim != 3) return fail(h, PASE_E_UNSUPPORTED, "3D only");
  if (h->fine_general) return fail(h, PASE_E_UNSUPPORTED, "the tensor-coefficient problem has no log kappa");
  launch_node_logk(h->lev[0].n, h->kappa, logk, h->stream);
  HIPC(hipGetLastError());
  HIPC(hipStreamSynchronize(h->stream));
  return PASE_OK;
}

pase_status pase_time_kernel(pase_handle* h, int which, int k, int reps, double* ms) {
  pase_status st = check_k(h, k);
  if (st) return st;
  if (!ms || reps < 1 || which < 0 || which > 7 || which == 4) return fail(h, PASE_E_ARG, "bad timing arguments");
  hipStream_t s = h->stream;
  const long long N = h->lev[0].N;
  auto once = [&]() {
    switch (which) {
      case 0: stencil_op(h, 0, k, EPI_SWEEP, h->U, h->R, h->Z, nullptr); break;
      case 1: apply_AM(h, 0, k, h->U, h->W2, h->W3); break;
      case 2: launch_gram(N, k, h->U, h->W2, h->partial, gram_tiles(N, k), h->kk1, s); break;
      case 3: vcycle(h, 0, k, h->R, h->Z); break;
      case 5: launch_axpy2(N, k, h->alpha, h->P, h->Q, h->W2, h->W3, s); break;   // on scratch
      case 6: apply_AM(h, 0, k, h->U, h->W2, nullptr); break;
      case 7: apply_AM(h, 0, k, h->U, nullptr, h->W3); break;
    }
  };
  once();   // warm
  HIPC(hipEventRecord(h->ev0, s));
  for (int r = 0; r < reps; ++r) once();
  HIPC(hipEventRecord(h->ev1, s));
  HIPC(hipGetLastError());
  HIPC(hipEventSynchronize(h->ev1));
  float t = 0.f;
  HIPC(hipEventElapsedTime(&t, h->ev0, h->ev1));
  *ms = (double)t / reps;
  return PASE_OK;
}

}  // extern "C"
