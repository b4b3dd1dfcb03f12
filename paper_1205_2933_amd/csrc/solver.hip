// Solvers: minimal-residual smoother, coarse CGNE, the two-level V-cycle,
// flexible GCR with FP64 iterative refinement, the adaptive setup and the CGNE
// control.  Host code that enqueues kernels on the handle's stream; scalars
// stay on the device (slot table, see vecops.h) and the host reads them only
// for stopping tests.
//
// Paper: Sec. 2 (V-cycle in five steps; adaptive setup on A x = 0; coarse
// blocks over the whole fifth dimension), Sec. 3 (flexible GCR outer solver;
// cost counted in fine-operator applications; CG on the squared operator as
// the control).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <initializer_list>
#include <type_traits>
#include <vector>

#include "ctx.h"
#include "solver.h"

namespace mgdwf {

namespace {

// slot table (per right-hand side)
constexpr int S_CRR0 = 2, S_CRR_A = 3, S_CRR_B = 4, S_CPP = 5;    // coarse CGNE
constexpr int S_DOT = 8;                                          // multidot block (<= 16 dots + 3)
constexpr int S_QN = 48;                                          // |q_k|^2 at S_QN+k, <q_k, r> after it
constexpr int S_RIN = 70, S_R64 = 71, S_B = 72, S_TMP = 73;       // FGCR residuals
constexpr int S_GRR_A = 80, S_GRR_B = 81, S_GPAP = 82;            // CG on the normal equations
constexpr int S_SQ = 84;                                          // squared smoother: |p|^2, <p, r>
constexpr int S_CPQ = 88;                                         // coarse CG: |p|^2, <p, A_c p>
constexpr int S_MR = 96;                                          // MR step i: |p_i|^2, |q_i|^2 at S_MR + 2i, +1

template <class C2> struct Prec;
template <> struct Prec<double2> { static constexpr const char* tag = "64"; };
template <> struct Prec<float2> { static constexpr const char* tag = "32"; };

std::vector<double> read_slots(mgdwf_ctx* c, int nrhs) {
  std::vector<double> h((size_t)nrhs * NSLOT);
  double* sl = c->buf<double>("slots", (size_t)nrhs * NSLOT);
  MG_HIP(hipMemcpyAsync(h.data(), sl, h.size() * sizeof(double), hipMemcpyDeviceToHost, c->st));
  MG_HIP(hipStreamSynchronize(c->st));
  return h;
}

// Upload a table of device pointers (kept in a named workspace).
template <class C2>
const C2* const* ptr_table(mgdwf_ctx* c, const std::string& name, const std::vector<C2*>& ptrs) {
  const size_t before = c->ws.count(name) ? c->ws[name].bytes : 0;
  C2** d = c->buf<C2*>(name, std::max<size_t>(ptrs.size(), 1));
  // upload only when the table changed (or its buffer moved): the workspaces
  // behind the pointers are stable, so repeated V-cycles skip the copy and
  // the stream synchronisation it needs
  std::vector<void*> key(ptrs.begin(), ptrs.end());
  key.push_back(d);
  auto it = c->ptr_cache.find(name);
  if (it != c->ptr_cache.end() && it->second == key && before >= ptrs.size() * sizeof(C2*)) return d;
  MG_HIP(hipMemcpyAsync(d, ptrs.data(), ptrs.size() * sizeof(C2*), hipMemcpyHostToDevice, c->st));
  MG_HIP(hipStreamSynchronize(c->st));
  c->ptr_cache[name] = std::move(key);
  return d;
}

// ---------------------------------------------------------------- fine ops
template <class F2> const F2* gauge_of(mgdwf_ctx* c);
template <> const double2* gauge_of<double2>(mgdwf_ctx* c) { return c->U64.as<double2>(); }
template <> const float2* gauge_of<float2>(mgdwf_ctx* c) { return c->U32.as<float2>(); }
template <class F2> const F2* basis_of(mgdwf_ctx* c);
template <> const double2* basis_of<double2>(mgdwf_ctx* c) { return c->V64.as<double2>(); }
template <> const float2* basis_of<float2>(mgdwf_ctx* c) { return c->V32.as<float2>(); }

// out = D in (or D^+, or b - D in); optional |out|^2 into slot `dst`.
template <class F2>
void fine_op(mgdwf_ctx* c, const F2* in, F2* out, const F2* b, bool dag, int mode, int nrhs, int dst) {
  double* partial = nullptr;
  const int nb = fine_nblocks<F2>(c, nrhs);
  if (dst >= 0) partial = c->buf<double>("dpart", (size_t)nb * nrhs);
  fine_dslash<F2>(c, in, out, b, dag, mode, nrhs, partial, c->st);
  if (dst >= 0) finalize_rhs(partial, nb, 1, c->buf<double>("slots", (size_t)nrhs * NSLOT), dst, nrhs, c->st);
  c->fine_applies += 1;
}

// |v|^2 (and <v, w>) into slots dst, dst+1..2
template <class C2>
void norm_into(mgdwf_ctx* c, const C2* v, const C2* w, long long n, int nrhs, int dst) {
  double* partial = c->buf<double>("vpart", (size_t)VEC_BLOCKS * nrhs * (2 * 16 + 3));
  multidot_rhs<C2>(nullptr, 0, v, w, n, nrhs, partial, c->buf<double>("slots", (size_t)nrhs * NSLOT), dst, c->st);
}

template <class C2>
void copy(mgdwf_ctx* c, const C2* in, C2* out, long long n) {
  MG_HIP(hipMemcpyAsync(out, in, n * sizeof(C2), hipMemcpyDeviceToDevice, c->st));
}

// y = D_c x or D_c^+ x in the precision the parameters select
inline void coarse_op(mgdwf_ctx* c, const mgdwf_mg_params&, const double2* x, double2* y, bool dag, int nrhs) {
  coarse_apply64(dag ? c->DcH : c->Dc, x, y, c->cg, nrhs, c->st);
  c->coarse_applies += 1;
}
inline void coarse_op(mgdwf_ctx* c, const mgdwf_mg_params& p, const float2* x, float2* y, bool dag, int nrhs) {
  coarse_apply32(dag ? c->DcH : c->Dc, p.coarse_prec, x, y, c->cg, nrhs,
                 c->buf<char>("vc_pack", coarse_pack_bytes(c->cg, nrhs)), c->g.ctile, c->st);
  c->coarse_applies += 1;
}

// ---------------------------------------------------------------- V-cycle
template <class F2>
struct TwoLevel {
  mgdwf_ctx* c;
  int nrhs;
  mgdwf_mg_params p;
  long long nf, nc;  // per-RHS lengths (complex numbers)
  F2 *r1, *qq, *b3, *r3;
  F2 *cb, *cx, *cr, *cp, *cq, *ct;  // coarse vectors (same real type as the fine level)
  double* sl;
  double* vpart;

  TwoLevel(mgdwf_ctx* ctx, int n_rhs, const mgdwf_mg_params& prm) : c(ctx), nrhs(n_rhs), p(prm) {
    nf = c->fine_len();
    nc = c->coarse_len();
    const std::string t = Prec<F2>::tag;
    r1 = c->buf<F2>("vc_r1" + t, nf * nrhs);
    qq = c->buf<F2>("vc_q" + t, nf * nrhs);
    b3 = c->buf<F2>("vc_b3" + t, nf * nrhs);
    r3 = c->buf<F2>("vc_r3" + t, nf * nrhs);
    cb = c->buf<F2>("vc_cb" + t, nc * nrhs);
    cx = c->buf<F2>("vc_cx" + t, nc * nrhs);
    cr = c->buf<F2>("vc_cr" + t, nc * nrhs);
    cp = c->buf<F2>("vc_cp" + t, nc * nrhs);
    cq = c->buf<F2>("vc_cq" + t, nc * nrhs);
    ct = c->buf<F2>("vc_ct" + t, nc * nrhs);
    sl = c->buf<double>("slots", (size_t)nrhs * NSLOT);
    vpart = c->buf<double>("vpart", (size_t)VEC_BLOCKS * nrhs * (2 * 16 + 3));
  }

  // nu steps of minimal residual along D^+ r on D x = b from x = 0.  The
  // directions p_i are kept and x = sum_i alpha_i p_i is formed once at the end
  // (with smoother_dirs = k, at most k are kept and added to x every k
  // steps), so a step moves r, q and the new r only; step 0 reads b in place
  // of r.  Without need_r the last step skips the residual update nobody
  // reads; with add_x the step sum is added to x instead of replacing it.
  void smooth(const F2* b, F2* x, F2* r, int nu, bool need_r = true, bool add_x = false) {
    if (nu == 0) {
      copy(c, b, r, nf * nrhs);
      if (!add_x) zero<F2>(x, nf * nrhs, c->st);
      return;
    }
    const std::string t = Prec<F2>::tag;
    const int K = p.smoother_dirs > 0 ? std::min(nu, p.smoother_dirs) : nu;  // directions kept at once
    std::vector<F2*> P(K);
    for (int i = 0; i < K; ++i) P[i] = c->buf<F2>("mr_p" + std::to_string(i) + t, nf * nrhs);
    // one table per number kept: with nu_pre != nu_post a shared table would
    // be re-uploaded (with a stream synchronisation) inside captures
    const F2* const* Pd = ptr_table<F2>(c, "ptrP" + t + std::to_string(K), P);
    for (int i = 0; i < nu; ++i) {
      const F2* rin = i == 0 ? b : r;
      F2* pi = P[i % K];
      fine_op<F2>(c, rin, pi, nullptr, true, 0, nrhs, S_MR + 2 * i);       // p_i = D^+ r, |p_i|^2
      fine_op<F2>(c, pi, qq, nullptr, false, 0, nrhs, S_MR + 2 * i + 1);   // q = D p_i, |q|^2
      if (need_r || i + 1 < nu) res_update<F2>(r, rin, qq, nf, nrhs, sl, S_MR + 2 * i, S_MR + 2 * i + 1, c->st);
      if ((i + 1) % K == 0 || i + 1 == nu) {  // x (+)= sum of the kept directions' steps
        const int i0 = i - i % K;
        lincomb<F2>(x, Pd, i - i0 + 1, nf, nrhs, sl, S_MR + 2 * i0, add_x || i0 > 0, c->st);
      }
    }
  }

  // CGNE on D_c: x = D_c^+ y with D_c D_c^+ y = b, to |r| < tol |b| or maxiter.
  // Convergence is tested on the host every `check` iterations.  With
  // p.coarse_graph, every block of `check` iterations after the first is one
  // replay of a HIP graph captured from the same launches (their arguments
  // are the same in every block: the slot pair swaps an even number of times).
  static constexpr int check = 8;

  void cg_iteration(F2* x, int it, int cur, int nxt) {
    coarse_op(c, p, cp, cq, false, nrhs);
    mr_update<F2>(x, cr, cp, cq, nc, nrhs, sl, cur, S_CPP, it == 0, vpart, c->st);
    finalize_rhs(vpart, vec_blocks(nc), 1, sl, nxt, nrhs, c->st);
    coarse_op(c, p, cr, ct, true, nrhs);
    cg_dir<F2>(cp, ct, nc, nrhs, sl, nxt, cur, vpart, c->st);
    finalize_rhs(vpart, vec_blocks(nc), 1, sl, S_CPP, nrhs, c->st);
  }

  // Capture `body` (launches only, no host synchronisation, every workspace
  // already allocated) as a graph on the private stream; nothing runs now and
  // replays go to c->st.  The operator-application counters the body bumps are
  // kept per graph and added at each replay.
  template <class Body>
  mgdwf_ctx::Graph& capture(const std::string& key, Body&& body) {
    mgdwf_ctx::Graph& gr = c->graphs[key];
    if (gr.exec) return gr;
    if (!c->cap_st) MG_HIP(hipStreamCreateWithFlags(&c->cap_st, hipStreamNonBlocking));
    hipStream_t saved = c->st;
    const long long fa = c->fine_applies, ca = c->coarse_applies;
    c->st = c->cap_st;
    hipGraph_t graph = nullptr;
    MG_HIP(hipStreamBeginCapture(c->st, hipStreamCaptureModeThreadLocal));
    try {
      body();
    } catch (...) {
      (void)hipStreamEndCapture(c->st, &graph);
      if (graph) (void)hipGraphDestroy(graph);
      c->st = saved;
      c->fine_applies = fa;
      c->coarse_applies = ca;
      c->graphs.erase(key);
      throw;
    }
    MG_HIP(hipStreamEndCapture(c->st, &graph));
    c->st = saved;
    gr.fine = c->fine_applies - fa;
    gr.coarse = c->coarse_applies - ca;
    c->fine_applies = fa;
    c->coarse_applies = ca;
    hipGraphExec_t exec = nullptr;
    const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) c->graphs.erase(key);
    MG_HIP(e);
    gr.exec = exec;
    return gr;
  }

  void replay(const mgdwf_ctx::Graph& gr) {
    MG_HIP(hipGraphLaunch(gr.exec, c->st));
    c->fine_applies += gr.fine;
    c->coarse_applies += gr.coarse;
  }

  // Run `body` through a graph under `key` when graphs are enabled: eagerly the
  // first time (allocating its workspaces and uploading its pointer tables),
  // captured and replayed from the second time on.
  template <class Body>
  void segment(const std::string& key, Body&& body) {
    if (!p.coarse_graph) {
      body();
      return;
    }
    auto it = c->graphs.find(key);
    if (it == c->graphs.end()) {
      body();
      c->graphs[key];  // seen once
      return;
    }
    replay(capture(key, body));
  }

  std::string key_of(const char* what, std::initializer_list<const void*> ptrs) const {
    std::string k = std::string(what) + Prec<F2>::tag + ":" + std::to_string(nrhs) + ":" +
                    std::to_string((int)p.coarse_prec) + ":" + std::to_string(c->g.ftile) + ":" +
                    std::to_string(c->g.ctile) + ":" + std::to_string(p.nu_pre) + ":" + std::to_string(p.nu_post) +
                    ":" + std::to_string(c->ws_gen);
    char buf[32];
    for (const void* q : ptrs) {
      snprintf(buf, sizeof buf, ":%p", q);
      k += buf;
    }
    return k;
  }

  // one block of `check` coarse CGNE iterations (their arguments are the same
  // in every block: the slot pair swaps an even number of times)
  const mgdwf_ctx::Graph& block_graph(F2* x) {
    const CoarseStore& s1 = c->Dc;
    const CoarseStore& s2 = c->DcH;
    const std::string key = key_of("cg", {x, cr, cp, cq, ct, sl, vpart, s1.m64.p, s1.m32.p, s1.re16.p, s1.reb.p,
                                          s2.m64.p, s2.m32.p, s2.re16.p, s2.reb.p});
    return capture(key, [&] {
      int cur = S_CRR_A, nxt = S_CRR_B;
      for (int k = 0; k < check; ++k) {
        cg_iteration(x, 1, cur, nxt);
        std::swap(cur, nxt);
      }
    });
  }

  void coarse_solve(const F2* b, F2* x) {
    if (p.coarse_graph == 2) {
      if constexpr (std::is_same<F2, float2>::value) {
        char* work = c->buf<char>("cg_persist", persistent_cgne_bytes(c->cg, nrhs));
        if (coarse_cgne_persistent(c->Dc, c->DcH, p.coarse_prec, b, x, cr, cp, work,
                                   c->buf<long long>("cg_count", 1), c->cg, nrhs, p.coarse_tol, p.coarse_maxiter,
                                   c->barrier_wait_s, c->device, c->st)) {
          if (persistent_cgne_error(work, c->cg, nrhs, c->st))
            fail(MGDWF_ERR_HIP, "persistent coarse solve: a grid barrier wait ran out of time");
          return;
        }
      }
      ++c->persist_fallbacks;  // not applicable here: the launched loop below
    }
    copy(c, b, cr, nc * nrhs);
    norm_into<F2>(c, cr, nullptr, nc, nrhs, S_CRR0);
    norm_into<F2>(c, cr, nullptr, nc, nrhs, S_CRR_A);
    coarse_op(c, p, cr, cp, true, nrhs);
    norm_into<F2>(c, cp, nullptr, nc, nrhs, S_CPP);
    int cur = S_CRR_A, nxt = S_CRR_B;
    const double tol2 = p.coarse_tol * p.coarse_tol;
    int it = 0;
    while (it < p.coarse_maxiter) {
      if (p.coarse_graph && it > 0 && it % check == 0 && it + check <= p.coarse_maxiter) {
        replay(block_graph(x));
        it += check;  // cur and nxt are back where they were
      } else {
        cg_iteration(x, it, cur, nxt);
        std::swap(cur, nxt);
        ++it;
      }
      if (it % check == 0 && it < p.coarse_maxiter) {
        std::vector<double> h = read_slots(c, nrhs);
        bool done = true;
        for (int r = 0; r < nrhs; ++r)
          if (!(h[r * NSLOT + cur] <= tol2 * h[r * NSLOT + S_CRR0])) done = false;
        if (done) break;
      }
    }
  }

  // z = M b (the five steps of the paper's V-cycle)
  // The launches before and after the coarse solve have no host
  // synchronisation; with p.coarse_graph each runs as one graph replay.
  void apply(const F2* b, F2* z) {
    const F2* V = basis_of<F2>(c);
    c->phase_mark(0);
    segment(key_of("pre", {b, z, V, gauge_of<F2>(c)}), [&] {
      smooth(b, z, r1, p.nu_pre);                                        // x1 = S1^nu1(A, b), r1 = b - A x1
      restrict_op<F2, F2>(V, r1, cb, c->buf<double>("rpart", restrict_partial_doubles(c->cg, nrhs)), c->g, c->cg,
                          nrhs, c->st);                                  // b2 = R r1
    });
    c->phase_mark(1);
    coarse_solve(cb, cx);                                                // x2 = S2(RAP, b2)
    c->phase_mark(2);
    segment(key_of("post", {b, z, V, gauge_of<F2>(c)}), [&] {
      prolong_op<F2, F2>(V, cx, z, true, c->g, c->cg, nrhs, c->st);     // x1 + P x2
      if (p.nu_post > 0) {
        fine_op<F2>(c, z, b3, b, false, 1, nrhs, -1);                    // b3 = b - A(P x2 + x1)
        smooth(b3, z, r3, p.nu_post, false, true);                       // z += S3^nu3(A, b3)
      }
    });
    c->phase_mark(3);
  }
};

// ---------------------------------------------------------------- squared V-cycle
// The multigrid on N = D^+ D that the paper ran (Sec. 3, first paragraph;
// Sec. 4): z = M b = V(D^+ b), V the five-step V-cycle of Sec. 2 on N with
// minimal-residual smoothing on N, the Galerkin coarse operator
// A_c = P^+ N P (33-point, Hermitian) solved by CG, and the residual after
// the coarse correction recomputed with N.  M approximates N^-1 D^+ = D^-1,
// so it preconditions the same flexible GCR on D x = b.
inline void sq_op(mgdwf_ctx* c, const double2* x, double2* y, int nrhs) {
  sq_apply64(c->Asq.m64.as<double2>(), x, y, c->cg, nrhs, c->st);
  c->coarse_applies += 1;
}
inline void sq_op(mgdwf_ctx* c, const float2* x, float2* y, int nrhs) {
  sq_apply32(c->Asq.m32.as<float2>(), x, y, c->cg, nrhs, c->st);
  c->coarse_applies += 1;
}

inline void l2_op(mgdwf_ctx* c, const double2* x, double2* y, int nrhs) {
  sq_apply64(c->Acc64.as<double2>(), x, y, c->cg2, nrhs, c->st);
  c->coarse_applies += 1;
}
inline void l2_op(mgdwf_ctx* c, const float2* x, float2* y, int nrhs) {
  sq_apply32(c->Acc32.as<float2>(), x, y, c->cg2, nrhs, c->st);
  c->coarse_applies += 1;
}
template <class F2> const F2* l2_basis(mgdwf_ctx* c);
template <> const double2* l2_basis<double2>(mgdwf_ctx* c) { return c->W2_64.as<double2>(); }
template <> const float2* l2_basis<float2>(mgdwf_ctx* c) { return c->W2_32.as<float2>(); }

template <class F2>
struct TwoLevelSq {
  mgdwf_ctx* c;
  int nrhs;
  mgdwf_mg_params p;
  long long nf, nc;
  F2 *g, *ra, *rb, *t, *q, *r1, *r3;
  F2 *cb, *cx, *cr, *cp, *cq;
  double* sl;
  double* vpart;

  TwoLevelSq(mgdwf_ctx* ctx, int n_rhs, const mgdwf_mg_params& prm) : c(ctx), nrhs(n_rhs), p(prm) {
    nf = c->fine_len();
    nc = c->coarse_len();
    const std::string tg = Prec<F2>::tag;
    g = c->buf<F2>("sq_g" + tg, nf * nrhs);
    ra = c->buf<F2>("sq_ra" + tg, nf * nrhs);
    rb = c->buf<F2>("sq_rb" + tg, nf * nrhs);
    t = c->buf<F2>("sq_t" + tg, nf * nrhs);
    q = c->buf<F2>("sq_q" + tg, nf * nrhs);
    r1 = c->buf<F2>("sq_r1" + tg, nf * nrhs);
    r3 = c->buf<F2>("sq_r3" + tg, nf * nrhs);
    cb = c->buf<F2>("sq_cb" + tg, nc * nrhs);
    cx = c->buf<F2>("sq_cx" + tg, nc * nrhs);
    cr = c->buf<F2>("sq_cr" + tg, nc * nrhs);
    cp = c->buf<F2>("sq_cp" + tg, nc * nrhs);
    cq = c->buf<F2>("sq_cq" + tg, nc * nrhs);
    sl = c->buf<double>("slots", (size_t)nrhs * NSLOT);
    vpart = c->buf<double>("vpart", (size_t)VEC_BLOCKS * nrhs * (2 * 16 + 3));
  }

  // nu minimal-residual steps on N x = f along the residual itself (q = N r,
  // alpha = <q, r>/|q|^2), x from 0 or added to (add_x); the last residual
  // goes to rout (which must differ from f and from ra, rb) unless rout is
  // null.  Two applications of D per step.
  void smooth(const F2* f, F2* x, F2* rout, int nu, bool add_x) {
    const F2* rin = f;
    for (int i = 0; i < nu; ++i) {
      fine_op<F2>(c, rin, t, nullptr, false, 0, nrhs, -1);  // t = D r
      fine_op<F2>(c, t, q, nullptr, true, 0, nrhs, -1);     // q = D^+ t = N r
      norm_into<F2>(c, q, rin, nf, nrhs, S_SQ);             // |q|^2, <q, r>
      F2* rnew = (i + 1 == nu && rout) ? rout : (rin == ra ? rb : ra);
      mrh_update<F2>(x, rnew, rin, q, nf, nrhs, sl, S_SQ + 1, S_SQ, i == 0 && !add_x, c->st);
      rin = rnew;
    }
  }

  // CG from x = 0 on the Hermitian operator op (vectors of n per RHS), to
  // |r| <= tol |b| tested every 8 iterations, or maxiter; r, p, q: workspaces
  template <class Op>
  void cg(Op op, const F2* b, F2* x, long long n, F2* r, F2* pv, F2* qv, double tol, int maxiter) {
    copy(c, b, r, n * nrhs);
    copy(c, b, pv, n * nrhs);
    norm_into<F2>(c, r, nullptr, n, nrhs, S_CRR0);
    norm_into<F2>(c, r, nullptr, n, nrhs, S_CRR_A);
    int cur = S_CRR_A, nxt = S_CRR_B;
    const double tol2 = tol * tol;
    double* part = c->buf<double>("vpart", (size_t)VEC_BLOCKS * nrhs * (2 * 16 + 3));
    for (int it = 0; it < maxiter;) {
      op(pv, qv);                                                           // q = A p
      norm_into<F2>(c, pv, qv, n, nrhs, S_CPQ);                             // <p, q> at S_CPQ + 1
      mr_update<F2>(x, r, pv, qv, n, nrhs, sl, cur, S_CPQ + 1, it == 0, part, c->st);  // x += a p, r -= a q
      finalize_rhs(part, vec_blocks(n), 1, sl, nxt, nrhs, c->st);           // |r|^2
      cg_dir<F2>(pv, r, n, nrhs, sl, nxt, cur, nullptr, c->st);             // p = r + beta p
      std::swap(cur, nxt);
      ++it;
      if (it % 8 == 0 && it < maxiter) {
        std::vector<double> h = read_slots(c, nrhs);
        bool done = true;
        for (int rr = 0; rr < nrhs; ++rr)
          if (!(h[rr * NSLOT + cur] <= tol2 * h[rr * NSLOT + S_CRR0])) done = false;
        if (done) break;
      }
    }
  }

  // ---- third level (a level-2 basis is installed and gamma > 0): the coarse
  // solve is gamma sweeps of e <- e + K2(b - A_c e), K2 the level-2 cycle
  F2 *e2 = nullptr, *f2 = nullptr, *s2a = nullptr, *s2b = nullptr, *s2r = nullptr, *s2q = nullptr;
  F2 *c3b = nullptr, *c3x = nullptr, *c3r = nullptr, *c3p = nullptr, *c3q = nullptr;
  long long n3 = 0;

  void l2_buffers() {
    if (e2) return;
    const std::string tg = Prec<F2>::tag;
    n3 = (long long)c->cg2.Vc * c->cg2.n2;
    e2 = c->buf<F2>("l2_e" + tg, nc * nrhs);
    f2 = c->buf<F2>("l2_f" + tg, nc * nrhs);
    s2a = c->buf<F2>("l2_sa" + tg, nc * nrhs);
    s2b = c->buf<F2>("l2_sb" + tg, nc * nrhs);
    s2r = c->buf<F2>("l2_sr" + tg, nc * nrhs);
    s2q = c->buf<F2>("l2_sq" + tg, nc * nrhs);
    c3b = c->buf<F2>("l3_b" + tg, n3 * nrhs);
    c3x = c->buf<F2>("l3_x" + tg, n3 * nrhs);
    c3r = c->buf<F2>("l3_r" + tg, n3 * nrhs);
    c3p = c->buf<F2>("l3_p" + tg, n3 * nrhs);
    c3q = c->buf<F2>("l3_q" + tg, n3 * nrhs);
  }

  // nu minimal-residual steps on A_c e = f along the residual (e from 0 or
  // added to); the last residual goes to rout unless it is null
  void smooth2(const F2* f, F2* e, F2* rout, int nu, bool add) {
    const F2* rin = f;
    for (int i = 0; i < nu; ++i) {
      sq_op(c, rin, s2q, nrhs);                                             // q = A_c r
      norm_into<F2>(c, s2q, rin, nc, nrhs, S_SQ);                           // |q|^2, <q, r>
      F2* rnew = (i + 1 == nu && rout) ? rout : (rin == s2a ? s2b : s2a);
      mrh_update<F2>(e, rnew, rin, s2q, nc, nrhs, sl, S_SQ + 1, S_SQ, i == 0 && !add, c->st);
      rin = rnew;
    }
  }

  // e = K2 f: smoothing on A_c, R2, CG on A_cc, P2, residual, smoothing
  void k2(const F2* f, F2* e) {
    const mgdwf_level2_params& q = c->l2p;
    const F2* W = l2_basis<F2>(c);
    const F2* r1 = f;
    if (q.nu > 0) {
      smooth2(f, e, s2r, q.nu, false);
      r1 = s2r;
    } else {
      zero<F2>(e, nc * nrhs, c->st);
    }
    restrict2<F2>(W, r1, c3b, c->cg, c->cg2, nrhs, c->st);
    cg([&](const F2* a, F2* b) { l2_op(c, a, b, nrhs); }, c3b, c3x, n3, c3r, c3p, c3q, q.coarse_tol,
       q.coarse_maxiter);
    prolong2<F2>(W, c3x, e, true, c->cg, c->cg2, nrhs, c->st);
    if (q.nu > 0) {
      sq_op(c, e, s2q, nrhs);
      sub_into<F2>(s2r, f, s2q, nc * nrhs, c->st);                           // f - A_c e
      smooth2(s2r, e, nullptr, q.nu, true);
    }
  }

  void coarse_solve3(const F2* b, F2* x) {
    l2_buffers();
    for (int g = 0; g < c->l2p.gamma; ++g) {
      if (g == 0) {
        k2(b, x);
      } else {
        sq_op(c, x, s2q, nrhs);
        sub_into<F2>(f2, b, s2q, nc * nrhs, c->st);                          // b - A_c x
        k2(f2, e2);
        add_to<F2, F2>(x, e2, nc * nrhs, c->st);
      }
    }
  }

  // CG on A_c x = b from x = 0, to |r| <= tol |b| tested every 8 iterations, or
  // maxiter; with a third level, the level-2 cycles instead
  void coarse_solve(const F2* b, F2* x) {
    if (c->have_l2 && c->l2p.gamma > 0) {
      coarse_solve3(b, x);
      return;
    }
    copy(c, b, cr, nc * nrhs);
    copy(c, b, cp, nc * nrhs);
    norm_into<F2>(c, cr, nullptr, nc, nrhs, S_CRR0);
    norm_into<F2>(c, cr, nullptr, nc, nrhs, S_CRR_A);
    int cur = S_CRR_A, nxt = S_CRR_B;
    const double tol2 = p.coarse_tol * p.coarse_tol;
    for (int it = 0; it < p.coarse_maxiter;) {
      sq_op(c, cp, cq, nrhs);                                               // q = A_c p
      norm_into<F2>(c, cp, cq, nc, nrhs, S_CPQ);                            // <p, q> at S_CPQ + 1
      mr_update<F2>(x, cr, cp, cq, nc, nrhs, sl, cur, S_CPQ + 1, it == 0, vpart, c->st);  // x += a p, r -= a q
      finalize_rhs(vpart, vec_blocks(nc), 1, sl, nxt, nrhs, c->st);          // |r|^2
      cg_dir<F2>(cp, cr, nc, nrhs, sl, nxt, cur, nullptr, c->st);           // p = r + beta p
      std::swap(cur, nxt);
      ++it;
      if (it % 8 == 0 && it < p.coarse_maxiter) {
        std::vector<double> h = read_slots(c, nrhs);
        bool done = true;
        for (int r = 0; r < nrhs; ++r)
          if (!(h[r * NSLOT + cur] <= tol2 * h[r * NSLOT + S_CRR0])) done = false;
        if (done) break;
      }
    }
  }

  void apply(const F2* b, F2* z) {
    const F2* V = basis_of<F2>(c);
    c->phase_mark(0);
    fine_op<F2>(c, b, g, nullptr, true, 0, nrhs, -1);                      // g = D^+ b
    if (p.nu_pre > 0) {
      smooth(g, z, r1, p.nu_pre, false);                                    // x1 = S1(N, g), r1 = g - N x1
    } else {
      copy(c, g, r1, nf * nrhs);
      zero<F2>(z, nf * nrhs, c->st);
    }
    fine_restrict<F2>(c, V, r1, cb, nrhs);                                // g2 = R r1
    c->phase_mark(1);
    coarse_solve(cb, cx);                                                   // x2 = CG(A_c, g2)
    c->phase_mark(2);
    fine_prolong<F2>(c, V, cx, z, true, nrhs);                              // x1 + P x2
    if (p.nu_post > 0) {
      fine_op<F2>(c, z, t, nullptr, false, 0, nrhs, -1);                    // g3 = g - N (x1 + P x2)
      fine_op<F2>(c, t, r3, g, true, 1, nrhs, -1);
      smooth(r3, z, nullptr, p.nu_post, true);                              // z += S3(N, g3)
    }
    c->phase_mark(3);
  }
};

// ---------------------------------------------------------------- FGCR cycle
// Up to `kmax` flexible GCR steps on D e = r (inner precision F2), e from 0.
// Stops early when every |r|^2 <= stop2[rhs].  Returns the steps taken.
//
// Only q is orthogonalised on the device.  The search directions follow as
// z~_k = z_k - sum_{i<k} g_ki z~_i with the Gram-Schmidt coefficients g_ki,
// and e = sum_k b_k z~_k with b_k = <q_k, r> / |q_k|^2; the host keeps the
// g and b it reads from the slot table anyway, and e is formed once at the
// end as sum_j c_j z_j over the unmodified z_j (c = T b, T the unit upper
// triangular map from z to z~).  Same iterates as updating z~ and e in place,
// without streaming z and e through every step.
template <class F2, class MG>
int fgcr_cycle(mgdwf_ctx* c, MG& M, F2* r, F2* e, int nrhs, int kmax, const std::vector<double>& stop2,
               std::vector<double>* rin2_out) {
  using cd = std::complex<double>;
  const long long nf = c->fine_len();
  const std::string t = Prec<F2>::tag;
  std::vector<F2*> Z(kmax), Q(kmax);
  for (int k = 0; k < kmax; ++k) {
    Z[k] = c->buf<F2>("gcr_z" + std::to_string(k) + t, nf * nrhs);
    Q[k] = c->buf<F2>("gcr_q" + std::to_string(k) + t, nf * nrhs);
  }
  const F2* const* Zd = ptr_table<F2>(c, "ptrZ" + t, Z);
  const F2* const* Qd = ptr_table<F2>(c, "ptrQ" + t, Q);
  double* sl = c->buf<double>("slots", (size_t)nrhs * NSLOT);
  double* vpart = c->buf<double>("vpart", (size_t)VEC_BLOCKS * nrhs * (2 * 16 + 3));
  // g[rhs][k][i] and b[rhs][k]
  std::vector<cd> g((size_t)nrhs * kmax * kmax, cd(0.0, 0.0)), bk((size_t)nrhs * kmax, cd(0.0, 0.0));
  auto take_g = [&](const std::vector<double>& h, int k) {  // coefficients of the pass just run
    for (int rr = 0; rr < nrhs; ++rr) {
      const double* hs = h.data() + (size_t)rr * NSLOT;
      for (int i = 0; i < k; ++i) {
        const double d = hs[S_QN + i];
        const double inv = d > 0.0 ? 1.0 / d : 0.0;
        g[((size_t)rr * kmax + k) * kmax + i] += cd(hs[S_DOT + 2 * i] * inv, hs[S_DOT + 2 * i + 1] * inv);
      }
    }
  };
  int k = 0;
  for (; k < kmax; ++k) {
    M.apply(r, Z[k]);                                           // z = M r
    fine_op<F2>(c, Z[k], Q[k], nullptr, false, 0, nrhs, -1);    // q = D z
    // classical Gram-Schmidt of q against q_0..q_{k-1}; a second pass only
    // where the first cancelled most of q (|q| fell below 1/sqrt 2 of its
    // norm before the pass), the usual twice-is-enough criterion
    for (int pass = 0; pass < 2 && k > 0; ++pass) {
      multidot_rhs<F2>(Qd, k, Q[k], nullptr, nf, nrhs, vpart, sl, S_DOT, c->st);  // |q|^2 before at S_DOT + 2k
      orth_update<F2>(Q[k], nullptr, Qd, nullptr, k, nf, nrhs, sl, S_DOT, S_QN, c->st);
      norm_into<F2>(c, Q[k], r, nf, nrhs, S_QN + k);            // |q_k|^2, <q_k, r>
      std::vector<double> h = read_slots(c, nrhs);
      take_g(h, k);
      if (pass == 1) break;
      bool again = false;
      for (int rr = 0; rr < nrhs; ++rr)
        if (!(h[rr * NSLOT + S_QN + k] >= 0.5 * h[rr * NSLOT + S_DOT + 2 * k])) again = true;
      if (!again) break;
      ++c->gs_repeats;
    }
    if (k == 0) norm_into<F2>(c, Q[k], r, nf, nrhs, S_QN + k);  // |q_0|^2, <q_0, r>
    gcr_update<F2>(nullptr, r, nullptr, Q[k], nf, nrhs, sl, S_QN + k + 1, S_QN + k, false, vpart, c->st);
    finalize_rhs(vpart, vec_blocks(nf), 1, sl, S_RIN, nrhs, c->st);
    std::vector<double> h = read_slots(c, nrhs);
    bool done = true;
    for (int rr = 0; rr < nrhs; ++rr) {
      const double* hs = h.data() + (size_t)rr * NSLOT;
      const double d = hs[S_QN + k];
      const double inv = d > 0.0 ? 1.0 / d : 0.0;
      bk[(size_t)rr * kmax + k] = cd(hs[S_QN + k + 1] * inv, hs[S_QN + k + 2] * inv);
      double v = hs[S_RIN];
      if (!std::isfinite(v)) fail(MGDWF_ERR_NUMERIC, "non-finite residual in flexible GCR");
      if (!(v <= stop2[rr])) done = false;
    }
    if (rin2_out) {
      rin2_out->resize(nrhs);
      for (int rr = 0; rr < nrhs; ++rr) (*rin2_out)[rr] = h[rr * NSLOT + S_RIN];
    }
    if (done) { ++k; break; }
  }
  // e = sum_j c_j z_j, c = T b with z~_k = sum_j T[j][k] z_j
  std::vector<double2> coef((size_t)nrhs * 16, make_double2(0.0, 0.0));
  std::vector<cd> T((size_t)k * k);
  for (int rr = 0; rr < nrhs; ++rr) {
    std::fill(T.begin(), T.end(), cd(0.0, 0.0));
    for (int kk = 0; kk < k; ++kk) {
      T[(size_t)kk * k + kk] = 1.0;
      for (int j = 0; j < kk; ++j) {
        cd acc = 0.0;
        for (int i = j; i < kk; ++i) acc += g[((size_t)rr * kmax + kk) * kmax + i] * T[(size_t)j * k + i];
        T[(size_t)j * k + kk] = -acc;
      }
    }
    for (int j = 0; j < k; ++j) {
      cd cj = 0.0;
      for (int kk = j; kk < k; ++kk) cj += T[(size_t)j * k + kk] * bk[(size_t)rr * kmax + kk];
      coef[(size_t)rr * 16 + j] = make_double2(cj.real(), cj.imag());
    }
  }
  double2* coef_d = c->buf<double2>("gcr_coef", (size_t)nrhs * 16);
  MG_HIP(hipMemcpyAsync(coef_d, coef.data(), coef.size() * sizeof(double2), hipMemcpyHostToDevice, c->st));
  lincomb_c<F2>(e, Zd, k, nf, nrhs, coef_d, c->st);
  MG_HIP(hipStreamSynchronize(c->st));  // the host coefficient buffer goes out of scope
  return k;
}

}  // namespace

// ---------------------------------------------------------------- public (C++) API

template <class F2, class MG>
static void solve_impl(mgdwf_ctx* c, double2* b64, double2* x64, int nrhs, const mgdwf_solve_params& sp,
                       mgdwf_solve_report* rep) {
  const long long nf = c->fine_len();
  c->buf<double>("slots", (size_t)nrhs * NSLOT);  // the slot table, sized for nrhs
  double2* r64 = c->buf<double2>("sol_r64", nf * nrhs);
  F2* rin = c->buf<F2>(std::string("sol_rin") + Prec<F2>::tag, nf * nrhs);
  F2* e = c->buf<F2>(std::string("sol_e") + Prec<F2>::tag, nf * nrhs);
  MG M(c, nrhs, c->mp);
  const long long fa0 = c->fine_applies, ca0 = c->coarse_applies, gs0 = c->gs_repeats, pf0 = c->persist_fallbacks;
  c->harvest_phases();
  const double ph0[3] = {c->phase_s[0], c->phase_s[1], c->phase_s[2]};
  long long* pcount = c->buf<long long>("cg_count", 1);  // applications made by persistent coarse solves
  MG_HIP(hipMemsetAsync(pcount, 0, sizeof(long long), c->st));
  auto t0 = std::chrono::steady_clock::now();
  norm_into<double2>(c, b64, nullptr, nf, nrhs, S_B);
  std::vector<double> h = read_slots(c, nrhs);
  std::vector<double> b2(nrhs);
  for (int r = 0; r < nrhs; ++r) {
    b2[r] = h[r * NSLOT + S_B];
    if (!std::isfinite(b2[r])) fail(MGDWF_ERR_NUMERIC, "non-finite right-hand side");
  }
  int outer = 0, restarts = 0;
  std::vector<double> rel(nrhs, 0.0);
  bool converged = false;
  const int restart = std::max(1, std::min<int>(sp.restart, 16));
  double best_prev = INFINITY;
  int stall = 0;
  uint32_t flags = 0;
  while (true) {
    fine_op<double2>(c, x64, r64, b64, false, 1, nrhs, S_R64);  // true residual, FP64
    h = read_slots(c, nrhs);
    converged = true;
    double worst = 0.0;
    for (int r = 0; r < nrhs; ++r) {
      double rr = h[r * NSLOT + S_R64];
      if (!std::isfinite(rr)) { flags |= 1u; fail(MGDWF_ERR_NUMERIC, "non-finite true residual"); }
      rel[r] = b2[r] > 0 ? std::sqrt(rr / b2[r]) : 0.0;
      if (!(rel[r] < sp.tol)) converged = false;
      worst = std::max(worst, rel[r]);
    }
    if (converged || outer >= sp.max_outer) break;
    if (worst >= 0.999 * best_prev) { if (++stall >= 3) { flags |= 2u; break; } } else stall = 0;
    best_prev = std::min(best_prev, worst);
    convert<double2, F2>(r64, rin, nf * nrhs, c->st);
    std::vector<double> stop2(nrhs);
    for (int r = 0; r < nrhs; ++r) stop2[r] = 0.25 * sp.tol * sp.tol * b2[r];
    int kmax = std::min(restart, sp.max_outer - outer);
    int k = fgcr_cycle<F2, MG>(c, M, rin, e, nrhs, kmax, stop2, nullptr);
    add_to<F2, double2>(x64, e, nf * nrhs, c->st);
    outer += k;
    ++restarts;
  }
  c->harvest_phases();
  {
    long long n = 0;
    MG_HIP(hipMemcpyAsync(&n, c->buf<long long>("cg_count", 1), sizeof n, hipMemcpyDeviceToHost, c->st));
    MG_HIP(hipStreamSynchronize(c->st));
    c->coarse_applies += n;
  }
  double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (c->gs_repeats > gs0) flags |= 4u;
  if (c->persist_fallbacks > pf0) flags |= 8u;
  if (rep)
    for (int r = 0; r < nrhs; ++r) {
      rep[r].outer_iters = outer;
      rep[r].restarts = restarts;
      rep[r].fine_applies = c->fine_applies - fa0;
      rep[r].coarse_applies = c->coarse_applies - ca0;
      rep[r].true_relres = rel[r];
      rep[r].seconds = secs;
      rep[r].flags = flags;
      for (int k = 0; k < 3; ++k) rep[r].phase_seconds[k] = c->phase_s[k] - ph0[k];
    }
  if (!converged) fail(MGDWF_ERR_NOT_CONVERGED, "solve did not reach the requested tolerance");
}

template <class F2, class MG>
static void vcycle_apply_impl(mgdwf_ctx* c, const double2* b64, double2* z64, int nrhs) {
  const long long n = c->fine_len() * nrhs;
  MG M(c, nrhs, c->mp);
  if constexpr (std::is_same<F2, double2>::value) {
    M.apply(b64, z64);
  } else {
    float2* b32 = c->buf<float2>("vca_b32", n);
    float2* z32 = c->buf<float2>("vca_z32", n);
    convert<double2, float2>(b64, b32, n, c->st);
    M.apply(b32, z32);
    convert<float2, double2>(z32, z64, n, c->st);
  }
}

void vcycle_apply(mgdwf_ctx* c, const double2* b64, double2* z64, int nrhs) {
  c->buf<double>("slots", (size_t)nrhs * NSLOT);
  const bool f64 = c->mp.fine_prec == MGDWF_F64;
  if (c->mp.squared) {
    if (f64) vcycle_apply_impl<double2, TwoLevelSq<double2>>(c, b64, z64, nrhs);
    else vcycle_apply_impl<float2, TwoLevelSq<float2>>(c, b64, z64, nrhs);
  } else {
    if (f64) vcycle_apply_impl<double2, TwoLevel<double2>>(c, b64, z64, nrhs);
    else vcycle_apply_impl<float2, TwoLevel<float2>>(c, b64, z64, nrhs);
  }
  c->harvest_phases();
}

void mg_solve(mgdwf_ctx* c, double2* b64, double2* x64, int nrhs, const mgdwf_solve_params& sp,
              mgdwf_solve_report* rep) {
  if (c->mp.fine_prec == MGDWF_F64) {
    if (c->mp.coarse_prec != MGDWF_F64) fail(MGDWF_ERR_INVALID_ARG, "an FP64 fine level needs an FP64 coarse level");
    if (c->mp.squared) solve_impl<double2, TwoLevelSq<double2>>(c, b64, x64, nrhs, sp, rep);
    else solve_impl<double2, TwoLevel<double2>>(c, b64, x64, nrhs, sp, rep);
  } else if (c->mp.fine_prec == MGDWF_F32) {
    if (c->mp.coarse_prec == MGDWF_F64) fail(MGDWF_ERR_INVALID_ARG, "an FP32 fine level takes an F32/F16/BF16 coarse level");
    if (c->mp.squared) solve_impl<float2, TwoLevelSq<float2>>(c, b64, x64, nrhs, sp, rep);
    else solve_impl<float2, TwoLevel<float2>>(c, b64, x64, nrhs, sp, rep);
  } else {
    fail(MGDWF_ERR_INVALID_ARG, "fine precision must be F64 or F32");
  }
}

// CG on D^+D x = 0 from x (nrhs vectors in place): the Krylov sweep of the
// setup.  With check > 0 each vector ends as the iterate, of those after every
// check iterations and after the last, with the smallest |D x| / |x| (the
// earliest on a tie).
static void cgnr_null(mgdwf_ctx* c, double2* x, int nrhs, int iters, int check) {
  const long long nf = c->fine_len();
  double* sl = c->buf<double>("slots", (size_t)nrhs * NSLOT);
  double* vpart = c->buf<double>("vpart", (size_t)VEC_BLOCKS * nrhs * (2 * 16 + 3));
  double2* r = c->buf<double2>("cg_r", nf * nrhs);
  double2* p = c->buf<double2>("cg_p", nf * nrhs);
  double2* t = c->buf<double2>("cg_t", nf * nrhs);
  double2* Ap = c->buf<double2>("cg_ap", nf * nrhs);
  double2* z = c->buf<double2>("cg_zero", nf * nrhs);
  zero<double2>(z, nf * nrhs, c->st);
  fine_op<double2>(c, x, t, nullptr, false, 0, nrhs, -1);
  fine_op<double2>(c, t, r, z, true, 1, nrhs, S_GRR_A);  // r = -D^+ D x
  copy(c, r, p, nf * nrhs);
  int cur = S_GRR_A, nxt = S_GRR_B;
  double2* best = check > 0 ? c->buf<double2>("cg_best", nf * nrhs) : nullptr;
  std::vector<double> best_q(nrhs, INFINITY);
  for (int i = 1; i <= iters; ++i) {
    fine_op<double2>(c, p, t, nullptr, false, 0, nrhs, S_GPAP);  // t = D p, <p, D^+D p> = |t|^2
    fine_op<double2>(c, t, Ap, nullptr, true, 0, nrhs, -1);
    mr_update<double2>(x, r, p, Ap, nf, nrhs, sl, cur, S_GPAP, false, vpart, c->st);
    finalize_rhs(vpart, vec_blocks(nf), 1, sl, nxt, nrhs, c->st);
    cg_dir<double2>(p, r, nf, nrhs, sl, nxt, cur, nullptr, c->st);
    std::swap(cur, nxt);
    if (check > 0 && (i % check == 0 || i == iters)) {
      fine_op<double2>(c, x, t, nullptr, false, 0, nrhs, S_TMP + 3);  // |D x|^2
      norm_into<double2>(c, x, nullptr, nf, nrhs, S_TMP);              // |x|^2
      std::vector<double> h = read_slots(c, nrhs);
      for (int k = 0; k < nrhs; ++k) {
        const double q = h[k * NSLOT + S_TMP + 3] / h[k * NSLOT + S_TMP];
        if (q < best_q[k] || (i == iters && best_q[k] == INFINITY)) {
          best_q[k] = q;
          copy(c, x + (long long)k * nf, best + (long long)k * nf, nf);
        }
      }
    }
  }
  if (check > 0 && iters > 0) copy(c, best, x, nf * nrhs);
}

static void normalise(mgdwf_ctx* c, double2* v, int nrhs) {
  const long long nf = c->fine_len();
  norm_into<double2>(c, v, nullptr, nf, nrhs, S_TMP);
  scale_by_rsqrt_slot<double2>(v, v, nf, nrhs, c->buf<double>("slots", (size_t)nrhs * NSLOT), S_TMP, c->st);
}

static double median_null_residual(mgdwf_ctx* c, double2* v, int nrhs) {
  const long long nf = c->fine_len();
  double2* t = c->buf<double2>("cg_t", nf * nrhs);
  fine_op<double2>(c, v, t, nullptr, false, 0, nrhs, S_TMP + 3);  // |D v|^2
  norm_into<double2>(c, v, nullptr, nf, nrhs, S_TMP);              // |v|^2 (+ two scratch slots)
  std::vector<double> h = read_slots(c, nrhs);
  std::vector<double> q(nrhs);
  for (int r = 0; r < nrhs; ++r) q[r] = std::sqrt(h[r * NSLOT + S_TMP + 3] / h[r * NSLOT + S_TMP]);
  std::sort(q.begin(), q.end());
  return nrhs % 2 ? q[nrhs / 2] : 0.5 * (q[nrhs / 2 - 1] + q[nrhs / 2]);
}

void install_basis(mgdwf_ctx* c, const int block[4], int nvec);  // capi.cpp
void build_coarse(mgdwf_ctx* c);                                 // capi.cpp
void build_coarse_squared(mgdwf_ctx* c);                         // capi.cpp

// Adaptive setup (paper Sec. 2): W holds nh internal FP64 fields on entry,
// nh = nvec / 2 (each paired with its reflection) or, for the squared
// operator, nh = nvec (the basis is the vectors themselves).
void mg_setup(mgdwf_ctx* c, const mgdwf_mg_params& p, double2* W, mgdwf_setup_report* rep) {
  const int nh = p.squared ? p.nvec : p.nvec / 2;
  const long long nf = c->fine_len();
  auto t0 = std::chrono::steady_clock::now();
  int nsw = 0;
  // The vectors are independent: their CG runs and sweeps take them in
  // groups, so the workspaces (six fields per vector for CG, about forty for
  // a V-cycle-preconditioned sweep) stay bounded on large lattices; every
  // per-vector sum is the same as in one batch.
  const double field_bytes = (double)nf * sizeof(double2);
  const int g0 = std::max(1, std::min(nh, std::min(4, (int)(48e9 / (6.0 * field_bytes)))));
  for (int k0 = 0; k0 < nh; k0 += g0)
    cgnr_null(c, W + (long long)k0 * nf, std::min(g0, nh - k0), p.sweep0_iters, p.sweep0_check);
  // the CG fields are not needed again: give them back before the basis and
  // the coarse operator are built (the build's peak on large lattices)
  for (const char* nm : {"cg_r", "cg_p", "cg_t", "cg_ap", "cg_zero", "cg_best"}) c->ws.erase(nm);
  ++c->ws_gen;
  normalise(c, W, nh);
  auto rebuild = [&]() {
    // basis fields: the nh vectors and their fifth-dimension reflections
    c->cg.Nv = p.nvec;
    c->V64.alloc(nf * p.nvec * sizeof(double2));
    if (p.squared) {
      copy(c, W, c->V64.as<double2>(), nf * p.nvec);
      install_basis(c, p.block, p.nvec);
      build_coarse_squared(c);
      return;
    }
    double2* V = c->V64.as<double2>();
    copy(c, W, V, nf * nh);
    reflect5<double2>(W, V + nf * nh, c->g, nh, c->st);
    install_basis(c, p.block, p.nvec);
    build_coarse(c);
  };
  rebuild();
  if (rep) rep->null_residual[nsw] = median_null_residual(c, W, nh);
  ++nsw;
  mgdwf_mg_params sweep = p;
  sweep.fine_prec = MGDWF_F64;
  sweep.coarse_prec = MGDWF_F64;
  for (int s = 1; s < p.sweeps; ++s) {
    // the multigrid applied to the same problem (Sec. 2, adaptive setup):
    // sweep_iters flexible-GCR steps with the current V-cycle on D x = 0 from
    // x = W, i.e. e from 0 on D e = -D W and then W <- W + e, so W keeps what
    // the current multigrid fails to remove; then normalise and rebuild
    const int gs = std::max(1, std::min(nh, (int)(64e9 / (40.0 * field_bytes))));
    for (int k0 = 0; k0 < nh; k0 += gs) {
      const int ng = std::min(gs, nh - k0);
      double2* Wg = W + (long long)k0 * nf;
      double2* r = c->buf<double2>("setup_r", nf * ng);
      double2* e = c->buf<double2>("setup_e", nf * ng);
      double2* z = c->buf<double2>("setup_zero", nf * ng);
      zero<double2>(z, nf * ng, c->st);
      fine_op<double2>(c, Wg, r, z, false, 1, ng, -1);  // r = 0 - D W
      std::vector<double> stop2(ng, -1.0);              // never met: exactly sweep_iters steps
      const int kmax = std::max(1, std::min(p.sweep_iters, 16));
      if (p.squared) {
        TwoLevelSq<double2> M(c, ng, sweep);
        fgcr_cycle<double2>(c, M, r, e, ng, kmax, stop2, nullptr);
      } else {
        TwoLevel<double2> M(c, ng, sweep);
        fgcr_cycle<double2>(c, M, r, e, ng, kmax, stop2, nullptr);
      }
      add_to<double2, double2>(Wg, e, nf * ng, c->st);
    }
    normalise(c, W, nh);
    rebuild();
    if (rep && nsw < 8) rep->null_residual[nsw] = median_null_residual(c, W, nh);
    ++nsw;
  }
  c->Vnull.alloc(nf * nh * sizeof(double2));
  copy(c, W, c->Vnull.as<double2>(), nf * nh);
  c->nnull = nh;
  c->mp = p;
  c->have_params = true;
  // the setup's work fields are large (several per vector): give them back
  for (auto it = c->ws.begin(); it != c->ws.end();) {
    if (it->first.rfind("cg_", 0) == 0 || it->first.rfind("setup_", 0) == 0 || it->first.rfind("dc_", 0) == 0 ||
        it->first.rfind("sq_", 0) == 0)
      it = c->ws.erase(it);
    else
      ++it;
  }
  if (rep) {
    rep->sweeps_done = nsw;
    rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
}

// CGNE control (paper Sec. 3): CG on D D^+ y = b, x = D^+ y, FP64.
// Third level under the squared coarse operator: near-null vectors of A_c by
// CG on A_c w = 0 (all starts at once), normalised; their chirality-split
// block basis; A_cc = R2 A_c P2.
static void require(bool cond, mgdwf_status code, const char* msg) {
  if (!cond) fail(code, msg);
}

void setup_level2(mgdwf_ctx* c, const mgdwf_level2_params& p, const double2* W0, double* null_residual) {
  require(c->have_coarse && c->coarse_kind == 1, MGDWF_ERR_STATE,
       "the third level needs the squared coarse operator (a squared setup or mgdwf_build_coarse_squared)");
  const CoarseGeometry& cg = c->cg;
  CoarseGeometry c2{};
  c2.bvol = 1;
  c2.Vc = 1;
  for (int m = 0; m < 4; ++m) {
    require(p.block[m] >= 1 && cg.Lc[m] % p.block[m] == 0, MGDWF_ERR_INVALID_ARG,
         "level-2 blocks must divide the coarse lattice");
    c2.block[m] = p.block[m];
    c2.Lc[m] = cg.Lc[m] / p.block[m];
    c2.bvol *= p.block[m];
    c2.Vc *= c2.Lc[m];
  }
  require(p.nvec >= 1 && p.nvec <= 32 && p.nvec <= c2.bvol * cg.Nv, MGDWF_ERR_INVALID_ARG,
       "level-2 nvec must be 1..32 and at most the rows of a block panel");
  require(p.null_iters >= 0 && p.nu >= 0 && p.coarse_maxiter >= 1 && p.gamma >= 0 && p.gamma <= 4 &&
           p.coarse_tol >= 0.0,
       MGDWF_ERR_INVALID_ARG, "bad level-2 parameters");
  c2.Nv = p.nvec;
  c2.n2 = 2 * p.nvec;
  c->have_l2 = false;
  c->clear_graphs();
  const int n = p.nvec;
  const long long nc = c->coarse_len();
  double* sl = c->buf<double>("slots", (size_t)n * NSLOT);
  double* vpart = c->buf<double>("vpart", (size_t)VEC_BLOCKS * n * (2 * 16 + 3));
  c->W2null.alloc((size_t)n * nc * sizeof(double2));
  double2* w = c->W2null.as<double2>();
  MG_HIP(hipMemcpyAsync(w, W0, (size_t)n * nc * sizeof(double2), hipMemcpyDeviceToDevice, c->st));
  double2* r = c->buf<double2>("l2s_r", n * nc);
  double2* pv = c->buf<double2>("l2s_p", n * nc);
  double2* q = c->buf<double2>("l2s_q", n * nc);
  const double2* Ac = c->Asq.m64.as<double2>();
  if (p.null_iters > 0) {  // CG on A_c w = 0 from w: r = -A_c w, p = r
    sq_apply64(Ac, w, q, cg, n, c->st);
    zero<double2>(r, n * nc, c->st);
    sub_into<double2>(r, r, q, n * nc, c->st);
    copy(c, r, pv, n * nc);
    norm_into<double2>(c, r, nullptr, nc, n, S_CRR_A);
    int cur = S_CRR_A, nxt = S_CRR_B;
    for (int it = 0; it < p.null_iters; ++it) {
      sq_apply64(Ac, pv, q, cg, n, c->st);                                   // q = A_c p
      norm_into<double2>(c, pv, q, nc, n, S_CPQ);                            // <p, q>
      mr_update<double2>(w, r, pv, q, nc, n, sl, cur, S_CPQ + 1, false, vpart, c->st);  // w += a p, r -= a q
      finalize_rhs(vpart, vec_blocks(nc), 1, sl, nxt, n, c->st);
      cg_dir<double2>(pv, r, nc, n, sl, nxt, cur, nullptr, c->st);
      std::swap(cur, nxt);
    }
    c->coarse_applies += p.null_iters + 1;
  }
  norm_into<double2>(c, w, nullptr, nc, n, S_TMP);
  scale_by_rsqrt_slot<double2>(w, w, nc, n, sl, S_TMP, c->st);
  if (null_residual) {  // median |A_c w| for the unit vectors
    sq_apply64(Ac, w, q, cg, n, c->st);
    norm_into<double2>(c, q, nullptr, nc, n, S_TMP);
    std::vector<double> h = read_slots(c, n);
    std::vector<double> v(n);
    for (int k = 0; k < n; ++k) v[k] = std::sqrt(h[k * NSLOT + S_TMP]);
    std::sort(v.begin(), v.end());
    *null_residual = n % 2 ? v[n / 2] : 0.5 * (v[n / 2 - 1] + v[n / 2]);
  }
  c->W2_64.alloc((size_t)n * nc * sizeof(double2));
  copy(c, w, c->W2_64.as<double2>(), n * nc);
  if (!orthonormalise_level2(c->W2_64.as<double2>(), cg, c2, c->buf<int>("l2s_err", 1), c->st))
    fail(MGDWF_ERR_NUMERIC, "a level-2 block panel of the near-null vectors is numerically rank deficient");
  c->W2_32.alloc((size_t)n * nc * sizeof(float2));
  convert<double2, float2>(c->W2_64.as<double2>(), c->W2_32.as<float2>(), n * nc, c->st);
  c->Acc64.alloc(sq_coarse_entries(c2) * sizeof(double2));
  double2* probes = c->buf<double2>("l2s_probe", (size_t)c2.n2 * nc);
  double2* applied = c->buf<double2>("l2s_applied", (size_t)c2.n2 * nc);
  double2* rr = c->buf<double2>("l2s_rr", (size_t)c2.n2 * c2.Vc * c2.n2);
  build_level2_op(Ac, c->W2_64.as<double2>(), c->Acc64.as<double2>(), probes, applied, rr, cg, c2, c->st);
  c->coarse_applies += c2.Vc;
  c->Acc32.alloc(sq_coarse_entries(c2) * sizeof(float2));
  sq_to_f32(c->Acc64.as<double2>(), c->Acc32.as<float2>(), c2, c->st);
  MG_HIP(hipStreamSynchronize(c->st));
  for (const char* nm : {"l2s_r", "l2s_p", "l2s_q", "l2s_probe", "l2s_applied", "l2s_rr"}) c->ws.erase(nm);
  ++c->ws_gen;
  c->cg2 = c2;
  c->l2p = p;
  c->have_l2 = true;
}

void cgne_solve(mgdwf_ctx* c, double2* b, double2* x, const mgdwf_solve_params& sp, mgdwf_solve_report* rep) {
  const long long nf = c->fine_len();
  const int nrhs = 1;
  double* sl = c->buf<double>("slots", (size_t)nrhs * NSLOT);
  double* vpart = c->buf<double>("vpart", (size_t)VEC_BLOCKS * nrhs * (2 * 16 + 3));
  double2* r = c->buf<double2>("cg_r", nf);
  double2* p = c->buf<double2>("cg_p", nf);
  double2* q = c->buf<double2>("cg_t", nf);
  const long long fa0 = c->fine_applies;
  auto t0 = std::chrono::steady_clock::now();
  norm_into<double2>(c, b, nullptr, nf, 1, S_B);
  fine_op<double2>(c, x, r, b, false, 1, 1, S_GRR_A);       // r = b - D x
  fine_op<double2>(c, r, p, nullptr, true, 0, 1, S_GPAP);   // p = D^+ r
  int cur = S_GRR_A, nxt = S_GRR_B;
  int it = 0;
  double rel = 1.0;
  const int check = 16;
  std::vector<double> h = read_slots(c, 1);
  const double bb = h[S_B];
  rel = bb > 0 ? std::sqrt(h[S_GRR_A] / bb) : 0.0;
  while (it < sp.max_outer && rel >= sp.tol) {
    fine_op<double2>(c, p, q, nullptr, false, 0, 1, -1);      // q = D p
    mr_update<double2>(x, r, p, q, nf, 1, sl, cur, S_GPAP, false, vpart, c->st);
    finalize_rhs(vpart, vec_blocks(nf), 1, sl, nxt, 1, c->st);
    double2* t = c->buf<double2>("cg_ap", nf);
    fine_op<double2>(c, r, t, nullptr, true, 0, 1, -1);       // t = D^+ r
    cg_dir<double2>(p, t, nf, 1, sl, nxt, cur, vpart, c->st);
    finalize_rhs(vpart, vec_blocks(nf), 1, sl, S_GPAP, 1, c->st);
    std::swap(cur, nxt);
    ++it;
    if (it % check == 0) {
      h = read_slots(c, 1);
      rel = std::sqrt(h[cur] / bb);
      if (!std::isfinite(rel)) fail(MGDWF_ERR_NUMERIC, "non-finite residual in CGNE");
    }
  }
  fine_op<double2>(c, x, r, b, false, 1, 1, S_R64);
  h = read_slots(c, 1);
  double tr = bb > 0 ? std::sqrt(h[S_R64] / bb) : 0.0;
  if (rep) {
    rep->outer_iters = it;
    rep->restarts = 0;
    rep->fine_applies = c->fine_applies - fa0;
    rep->coarse_applies = 0;
    rep->true_relres = tr;
    rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    rep->flags = 0;
    for (double& ph : rep->phase_seconds) ph = 0.0;
  }
  if (!(tr < sp.tol)) fail(MGDWF_ERR_NOT_CONVERGED, "CGNE did not reach the requested tolerance");
}

}  // namespace mgdwf
