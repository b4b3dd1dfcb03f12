// The library context behind an mgdwf_handle.
#pragma once

#include <map>
#include <string>
#include <vector>

#include "mg_internal.h"
#include "vecops.h"

struct mgdwf_ctx {
  // 0: the 4D SU(3) operator; 1: the 2D U(1) operator (g.L = {Lx, Ly, 1, 1},
  // V4 = Lx * Ly, two spins, layouts in u1_2d.hip)
  int model = 0;
  mgdwf::Geometry g{};
  mgdwf::CoarseGeometry fg{};  // 2D model: the fine lattice as a coarse-vector lattice (Nv = Ls, chirality = spin)
  double M5 = 0.0, mf = 0.0;
  hipStream_t st = nullptr;
  int device = 0;
  void* scratch = nullptr;  // device address of this GPU's static scratch array (no-allocation entry point)

  mgdwf::DevBuf U64, U32;  // links, FP64 and FP32 (the FP32 buffer: component major, site major, phase folded)
  bool have_gauge = false;

  mgdwf::CoarseGeometry cg{};
  bool have_basis = false, have_coarse = false;
  mgdwf::DevBuf V64, V32;    // orthonormal basis, Nv fields
  mgdwf::DevBuf Vnull;       // the near-null vectors the basis was built from (FP64, internal layout)
  int nnull = 0;             // how many: nvec/2 after a setup, nvec after set_nullvecs
  mgdwf::CoarseStore Dc, DcH;  // coarse operator and its adjoint stencil, all precisions
  mgdwf::CoarseStore Asq;      // squared-operator coarse operator (33 offsets; FP64 and FP32 copies)
  int coarse_kind = 0;         // which coarse operator is built: 0 the 9-point D_c, 1 the squared A_c
  // third level under the squared coarse operator (mgdwf_setup_level2)
  bool have_l2 = false;
  mgdwf_level2_params l2p{};
  mgdwf::CoarseGeometry cg2{};   // level-2 lattice: Lc = blocks, Vc, Nv = Nv2, n2, block = coarse sites per block
  mgdwf::DevBuf W2null, W2_64, W2_32, Acc64, Acc32;

  mgdwf_mg_params mp{};
  bool have_params = false;

  std::map<std::string, mgdwf::DevBuf> ws;  // named workspaces, grown on demand
  std::map<std::string, std::vector<void*>> ptr_cache;  // device pointer tables as last uploaded
  // Captured launch sequences (coarse iteration blocks, V-cycle segments),
  // keyed by what they read and write; exec == nullptr marks a sequence that
  // has run eagerly once (so its workspaces and pointer tables exist) and is
  // captured on its next use.  fine / coarse: operator applications per replay.
  struct Graph {
    hipGraphExec_t exec = nullptr;
    long long fine = 0, coarse = 0;
  };
  std::map<std::string, Graph> graphs;
  hipStream_t cap_st = nullptr;  // private stream the graphs are captured on
  long long ws_gen = 0;          // bumped whenever a workspace is (re)allocated

  void clear_graphs() {
    for (auto& kv : graphs)
      if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
    graphs.clear();
  }
  // V-cycle phase timing: events on st bracketing the three phases of the
  // last V-cycle (before pre-smoothing, after restriction, after the coarse
  // solve, after post-smoothing) and the seconds summed per phase so far.
  hipEvent_t phase_ev[4] = {};
  bool phase_pending = false;
  double phase_s[3] = {0.0, 0.0, 0.0};

  void phase_mark(int i) {
    if (!phase_ev[0])
      for (hipEvent_t& e : phase_ev) MG_HIP(hipEventCreate(&e));
    if (i == 0) harvest_phases();
    MG_HIP(hipEventRecord(phase_ev[i], st));
    if (i == 3) phase_pending = true;
  }
  // Add the last complete V-cycle's phase times (waits for its last event).
  void harvest_phases() {
    if (!phase_pending) return;
    phase_pending = false;
    MG_HIP(hipEventSynchronize(phase_ev[3]));
    for (int k = 0; k < 3; ++k) {
      float ms = 0.0f;
      MG_HIP(hipEventElapsedTime(&ms, phase_ev[k], phase_ev[k + 1]));
      phase_s[k] += 1e-3 * ms;
    }
  }

  ~mgdwf_ctx() {
    clear_graphs();
    if (cap_st) (void)hipStreamDestroy(cap_st);
    for (hipEvent_t e : phase_ev)
      if (e) (void)hipEventDestroy(e);
  }
  std::string err;

  long long fine_applies = 0;    // per right-hand side, since the last reset
  long long coarse_applies = 0;
  long long gs_repeats = 0;      // flexible-GCR steps that needed a second Gram-Schmidt pass
  long long persist_fallbacks = 0;  // coarse solves where the persistent kernel was asked for but did not apply
  double barrier_wait_s = 10.0;  // bound of one grid-barrier wait in the persistent coarse kernel

  // Workspace `name` with room for `count` elements of T (contents undefined).
  template <class T>
  T* buf(const std::string& name, size_t count) {
    mgdwf::DevBuf& b = ws[name];
    size_t need = count * sizeof(T);
    if (b.bytes < need) {
      b.alloc(need);
      ++ws_gen;
    }
    return b.as<T>();
  }
  long long fine_len() const { return (model == 0 ? 12LL : 2LL) * g.V5; }  // complex numbers per fine field
  long long coarse_len() const { return (long long)cg.Vc * cg.n2; }
};

namespace mgdwf {

// Fine-level operations of the handle's model (u1_2d.hip): the 4D kernels for
// model 0, the 2D ones for model 1.
void pack_field(const mgdwf_ctx* c, const double2* canon, double2* field, int nrhs);
void unpack_field(const mgdwf_ctx* c, const double2* field, double2* canon, int nrhs);
// allocates and fills U64 / U32 in the model's internal gauge layouts
void pack_gauge_field(mgdwf_ctx* c, const double2* canon);
// workgroups (partial sums per right-hand side) of fine_dslash with a partial buffer
template <class F2> int fine_nblocks(const mgdwf_ctx* c, int nrhs);
// out = D in (D^+ for dag); mode 1: out = b - D in; partial: per-workgroup |out|^2
template <class F2>
void fine_dslash(const mgdwf_ctx* c, const F2* in, F2* out, const F2* b, bool dag, int mode, int nrhs,
                 double* partial, hipStream_t st);
template <class F2> void fine_restrict(mgdwf_ctx* c, const F2* V, const F2* in, F2* out, int nrhs);
template <class F2> void fine_prolong(mgdwf_ctx* c, const F2* V, const F2* cc, F2* out, bool acc, int nrhs);
// chirality split + block orthonormalisation of the nvec fields in V64 on c->cg
bool fine_orthonormalise(mgdwf_ctx* c);
// A_c = P^+ D^+D P of the 2D model into c->Asq.m64 (allocated by the caller)
void build_sq_coarse_2d(mgdwf_ctx* c);

}  // namespace mgdwf
