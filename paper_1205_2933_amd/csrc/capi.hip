// extern "C" entry points (include/mgdwf.h): argument validation, layout
// conversion at the boundary, and conversion of C++ errors to status codes.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "ctx.h"
#include "solver.h"

using namespace mgdwf;

namespace {

thread_local std::string g_create_error;

// Static scratch for mgdwf_apply_coarse_noalloc: every GPU the library runs
// on holds one copy until the process ends.  In host code `scratch` names a
// host-side stand-in, not a device address: its address on each device is
// taken once per device with hipGetSymbolAddress (with that device current)
// and kept; only that address is ever handed to kernels or copies.
constexpr size_t kScratchBytes = (size_t)16 << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_addr;

void* scratch_address(int device) {  // `device` is the current device
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_addr.find(device);
  if (it != g_scratch_addr.end()) return it->second;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || p == nullptr) fail(MGDWF_ERR_HIP, "hipGetSymbolAddress of the scratch array failed");
  g_scratch_addr[device] = p;
  return p;
}

template <class F>
mgdwf_status guarded(mgdwf_ctx* c, F&& f) {
  try {
    f();
    return MGDWF_OK;
  } catch (const Error& e) {
    if (c) c->err = e.msg;
    else g_create_error = e.msg;
    return e.code;
  } catch (const std::exception& e) {
    if (c) c->err = e.what();
    else g_create_error = e.what();
    return MGDWF_ERR_HIP;
  }
}

void need(bool cond, mgdwf_status code, const char* msg) {
  if (!cond) fail(code, msg);
}

void check_prec_fine(mgdwf_prec p) {
  need(p == MGDWF_F64 || p == MGDWF_F32, MGDWF_ERR_INVALID_ARG, "fine precision must be F64 or F32");
}

CoarseGeometry make_coarse(const mgdwf_ctx* c, const int32_t block[4], int nvec) {
  const Geometry& g = c->g;
  CoarseGeometry cg{};
  cg.bvol = 1;
  cg.Vc = 1;
  for (int m = 0; m < 4; ++m) {
    need(block[m] >= 1 && g.L[m] % block[m] == 0, MGDWF_ERR_INVALID_ARG, "block must divide the lattice");
    cg.block[m] = block[m];
    cg.Lc[m] = g.L[m] / block[m];
    cg.bvol *= block[m];
    cg.Vc *= cg.Lc[m];
  }
  need(nvec >= 1 && nvec <= 32, MGDWF_ERR_INVALID_ARG, "nvec must be in 1..32");
  // dof of a block per chirality: Ls x (2 spins x 3 colours) in 4D, Ls x 1 spin in 2D
  need(nvec <= (c->model == 0 ? 6 : 1) * g.Ls * cg.bvol, MGDWF_ERR_INVALID_ARG,
       "nvec exceeds the block's dof per chirality");
  cg.Nv = nvec;
  cg.n2 = 2 * nvec;
  return cg;
}

// The squared coarse stencil needs block extents >= 2 along the lattice's
// directions (the 2D model's z and t extents are 1, and so are its blocks there).
void check_sq_blocks(const mgdwf_ctx* c, const int32_t block[4]) {
  for (int m = 0; m < 4; ++m) {
    if (c->model == 1 && m >= 2) continue;
    need(block[m] >= 2, MGDWF_ERR_INVALID_ARG, "the squared-operator coarse stencil needs block extents >= 2");
  }
}

// The calls that exist for the 4D operator only.
void need_4d(const mgdwf_ctx* c, const char* what) {
  if (c->model != 0) fail(MGDWF_ERR_INVALID_ARG, std::string(what) + " is not available for the 2D U(1) model");
}

void check_params(const mgdwf_ctx* c, const mgdwf_mg_params* p) {
  need(p != nullptr, MGDWF_ERR_INVALID_ARG, "null parameters");
  need(p->squared == 0 || p->squared == 1, MGDWF_ERR_INVALID_ARG, "squared must be 0 or 1");
  need(c->model == 0 || p->squared == 1, MGDWF_ERR_INVALID_ARG, "the 2D U(1) model runs the squared-operator multigrid");
  if (p->squared) {
    need(p->nvec >= 1, MGDWF_ERR_INVALID_ARG, "nvec must be >= 1");
    need(p->coarse_prec == MGDWF_F64 || p->coarse_prec == MGDWF_F32, MGDWF_ERR_INVALID_ARG,
         "the squared-operator coarse level runs in F64 or F32");
    check_sq_blocks(c, p->block);
  } else {
    need(p->nvec >= 2 && p->nvec % 2 == 0, MGDWF_ERR_INVALID_ARG, "nvec must be even (vectors are paired with their reflections)");
  }
  need(p->sweeps >= 1 && p->sweeps <= 8, MGDWF_ERR_INVALID_ARG, "sweeps must be in 1..8");
  need(p->sweep0_iters >= 0 && p->sweep_iters >= 1 && p->sweep0_check >= 0, MGDWF_ERR_INVALID_ARG,
       "bad sweep iteration counts");
  need(p->smoother_dirs >= 0, MGDWF_ERR_INVALID_ARG, "smoother_dirs must be >= 0");
  need(p->nu_pre >= 0 && p->nu_post >= 0 && p->nu_pre <= 16 && p->nu_post <= 16, MGDWF_ERR_INVALID_ARG,
       "bad smoother step counts");
  need(p->coarse_tol > 0 && p->coarse_tol < 1 && p->coarse_maxiter >= 1, MGDWF_ERR_INVALID_ARG,
       "bad coarse solver settings");
  check_prec_fine(p->fine_prec);
  need(p->coarse_prec >= MGDWF_F64 && p->coarse_prec <= MGDWF_BF16, MGDWF_ERR_INVALID_ARG, "bad coarse precision");
  need(p->coarse_graph >= 0 && p->coarse_graph <= 2, MGDWF_ERR_INVALID_ARG, "coarse_graph must be 0, 1 or 2");
  (void)make_coarse(c, p->block, p->nvec);
}

}  // namespace

namespace mgdwf {

// Orthonormalise the nvec FP64 fields already in c->V64 on the given blocks.
void install_basis(mgdwf_ctx* c, const int block[4], int nvec) {
  c->have_basis = false;
  c->have_coarse = false;
  c->have_l2 = false;
  c->cg = make_coarse(c, block, nvec);
  if (!fine_orthonormalise(c))
    fail(MGDWF_ERR_NUMERIC, "a block panel of the near-null vectors is numerically rank deficient");
  const long long n = c->fine_len() * nvec;
  c->V32.alloc(n * sizeof(float2));
  convert<double2, float2>(c->V64.as<double2>(), c->V32.as<float2>(), n, c->st);
  MG_HIP(hipStreamSynchronize(c->st));
  c->have_basis = true;
}

void build_coarse_squared(mgdwf_ctx* c) {
  need(c->have_basis, MGDWF_ERR_STATE, "no basis installed");
  const CoarseGeometry& cg = c->cg;
  check_sq_blocks(c, cg.block);
  const long long field = c->fine_len();
  c->have_coarse = false;
  c->Asq.m64.alloc(sq_coarse_entries(cg) * sizeof(double2));
  if (c->model == 1) {
    build_sq_coarse_2d(c);
    c->Asq.m32.alloc(sq_coarse_entries(cg) * sizeof(float2));
    sq_to_f32(c->Asq.m64.as<double2>(), c->Asq.m32.as<float2>(), cg, c->st);
    MG_HIP(hipStreamSynchronize(c->st));
    for (const char* nm : {"dc_probe", "dc_applied", "dc_tmp", "dc_rr"}) c->ws.erase(nm);
    ++c->ws_gen;
    c->coarse_kind = 1;
    c->have_l2 = false;
    c->have_coarse = true;
    return;
  }
  double2* work9 = c->buf<double2>("dc_work9", 9 * field);
  double2* zwork9 = c->buf<double2>("dc_zwork9", 9 * field);
  double2* cwork = c->buf<double2>("dc_cwork", 9LL * cg.Vc * cg.n2);
  double* partial = c->buf<double>("dc_partial", restrict_partial_doubles(cg, 9));
  build_sq_coarse_op(c->V64.as<double2>(), c->U64.as<double2>(), c->Asq.m64.as<double2>(), work9, zwork9, cwork,
                     partial, c->g, cg, c->M5, c->mf, c->st);
  c->Asq.m32.alloc(sq_coarse_entries(cg) * sizeof(float2));
  sq_to_f32(c->Asq.m64.as<double2>(), c->Asq.m32.as<float2>(), cg, c->st);
  MG_HIP(hipStreamSynchronize(c->st));
  c->ws.erase("dc_work9");
  c->ws.erase("dc_zwork9");
  c->coarse_kind = 1;
  c->have_l2 = false;
  c->have_coarse = true;
}

void build_coarse(mgdwf_ctx* c) {
  need_4d(c, "the 9-point coarse operator");
  need(c->have_basis, MGDWF_ERR_STATE, "no basis installed");
  const CoarseGeometry& cg = c->cg;
  const long long ndc = (long long)cg.Vc * 9 * cg.n2 * cg.n2;
  c->Dc.m64.alloc(ndc * sizeof(double2));
  double2* work9 = c->buf<double2>("dc_work9", 9 * c->fine_len());
  double2* cwork = c->buf<double2>("dc_cwork", 9LL * cg.Vc * cg.n2);
  double* partial = c->buf<double>("dc_partial", restrict_partial_doubles(cg, 9));
  build_coarse_op(c->V64.as<double2>(), c->U64.as<double2>(), c->Dc.m64.as<double2>(), work9, cwork, partial, c->g,
                  cg, c->M5, c->mf, c->st);
  finish_coarse_op(c->Dc, c->DcH, cg, c->st);
  MG_HIP(hipStreamSynchronize(c->st));
  // the build workspaces are large; give them back
  c->ws.erase("dc_work9");
  c->coarse_kind = 0;
  c->have_l2 = false;
  c->have_coarse = true;
}

}  // namespace mgdwf

namespace {

__global__ void k_dc_canonical(const double2* __restrict__ in, double2* __restrict__ out, long long nblk, int n2) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long tot = nblk * n2 * n2;
  if (i >= tot) return;
  long long blk = i / ((long long)n2 * n2);
  int rc = (int)(i - blk * n2 * n2);
  int row = rc / n2, col = rc % n2;
  out[i] = in[blk * n2 * n2 + (long long)col * n2 + row];
}

}  // namespace

extern "C" {

mgdwf_status mgdwf_create(const mgdwf_action* a, void* hip_stream, mgdwf_handle* out) {
  return guarded(nullptr, [&] {
    need(a != nullptr && out != nullptr, MGDWF_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    need(a->Ls >= 1, MGDWF_ERR_INVALID_ARG, "Ls must be >= 1");
    for (int m = 0; m < 4; ++m) {
      need(a->L[m] >= 2, MGDWF_ERR_INVALID_ARG, "every extent must be >= 2");
      need(a->bc[m] == 1 || a->bc[m] == -1, MGDWF_ERR_INVALID_ARG, "bc must be +1 or -1");
    }
    need(std::isfinite(a->M5) && std::isfinite(a->mf), MGDWF_ERR_INVALID_ARG, "non-finite M5 or mf");
    long long V4 = (long long)a->L[0] * a->L[1] * a->L[2] * a->L[3];
    need(V4 * a->Ls * 12 < (1LL << 31), MGDWF_ERR_INVALID_ARG, "lattice too large for 32-bit site indices");
    auto* c = new mgdwf_ctx();
    for (int m = 0; m < 4; ++m) { c->g.L[m] = a->L[m]; c->g.bc[m] = a->bc[m]; }
    c->g.Ls = a->Ls;
    c->g.V4 = (int)V4;
    c->g.V5 = (int)(V4 * a->Ls);
    c->M5 = a->M5;
    c->mf = a->mf;
    c->st = static_cast<hipStream_t>(hip_stream);
    if (hipGetDevice(&c->device) != hipSuccess) {
      delete c;
      fail(MGDWF_ERR_HIP, "no HIP device");
    }
    try {
      c->scratch = scratch_address(c->device);
    } catch (...) {
      delete c;
      throw;
    }
    *out = c;
  });
}

mgdwf_status mgdwf_create_2d(const mgdwf_action2d* a, void* hip_stream, mgdwf_handle* out) {
  return guarded(nullptr, [&] {
    need(a != nullptr && out != nullptr, MGDWF_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    need(a->Ls >= 1, MGDWF_ERR_INVALID_ARG, "Ls must be >= 1");
    for (int m = 0; m < 2; ++m) {
      need(a->L[m] >= 2, MGDWF_ERR_INVALID_ARG, "every extent must be >= 2");
      need(a->bc[m] == 1 || a->bc[m] == -1, MGDWF_ERR_INVALID_ARG, "bc must be +1 or -1");
    }
    need(std::isfinite(a->M5) && std::isfinite(a->mf), MGDWF_ERR_INVALID_ARG, "non-finite M5 or mf");
    const long long V2 = (long long)a->L[0] * a->L[1];
    need(V2 * a->Ls * 2 < (1LL << 31), MGDWF_ERR_INVALID_ARG, "lattice too large for 32-bit site indices");
    auto* c = new mgdwf_ctx();
    c->model = 1;
    c->g.L[0] = a->L[0];
    c->g.L[1] = a->L[1];
    c->g.L[2] = c->g.L[3] = 1;
    c->g.bc[0] = a->bc[0];
    c->g.bc[1] = a->bc[1];
    c->g.bc[2] = c->g.bc[3] = 1;
    c->g.Ls = a->Ls;
    c->g.V4 = (int)V2;
    c->g.V5 = (int)(V2 * a->Ls);
    // the fine lattice seen as a lattice of coarse-vector sites: [x2][spin][s]
    c->fg.Lc[0] = a->L[0];
    c->fg.Lc[1] = a->L[1];
    c->fg.Lc[2] = c->fg.Lc[3] = 1;
    for (int m = 0; m < 4; ++m) c->fg.block[m] = 1;
    c->fg.bvol = 1;
    c->fg.Vc = (int)V2;
    c->fg.Nv = a->Ls;
    c->fg.n2 = 2 * a->Ls;
    c->M5 = a->M5;
    c->mf = a->mf;
    c->st = static_cast<hipStream_t>(hip_stream);
    if (hipGetDevice(&c->device) != hipSuccess) {
      delete c;
      fail(MGDWF_ERR_HIP, "no HIP device");
    }
    try {
      c->scratch = scratch_address(c->device);
    } catch (...) {
      delete c;
      throw;
    }
    *out = c;
  });
}

mgdwf_status mgdwf_destroy(mgdwf_handle h) {
  if (!h) return MGDWF_OK;
  (void)hipStreamSynchronize(h->st);
  delete h;
  return MGDWF_OK;
}

const char* mgdwf_last_error(mgdwf_handle h) { return h ? h->err.c_str() : g_create_error.c_str(); }

mgdwf_status mgdwf_set_gauge(mgdwf_handle h, const double* U) {
  if (!h) return MGDWF_ERR_INVALID_ARG;
  return guarded(h, [&] {
    need(U != nullptr, MGDWF_ERR_INVALID_ARG, "null gauge field");
    pack_gauge_field(h, reinterpret_cast<const double2*>(U));
    MG_HIP(hipStreamSynchronize(h->st));
    h->have_gauge = true;
    h->have_basis = false;
    h->have_coarse = false;
  });
}

mgdwf_status mgdwf_apply_dwf(mgdwf_handle h, const double* in, double* out, int32_t dagger, mgdwf_prec prec,
                             int32_t nrhs) {
  if (!h) return MGDWF_ERR_INVALID_ARG;
  return guarded(h, [&] {
    need(in && out, MGDWF_ERR_INVALID_ARG, "null field");
    need(nrhs >= 1, MGDWF_ERR_INVALID_ARG, "nrhs must be >= 1");
    check_prec_fine(prec);
    need(h->have_gauge, MGDWF_ERR_STATE, "gauge field not set");
    const long long n = h->fine_len() * nrhs;
    double2* a = h->buf<double2>("io_a", n);
    double2* b = h->buf<double2>("io_b", n);
    pack_field(h, reinterpret_cast<const double2*>(in), a, nrhs);
    if (prec == MGDWF_F64) {
      fine_dslash<double2>(h, a, b, nullptr, dagger != 0, 0, nrhs, nullptr, h->st);
    } else {
      float2* a32 = h->buf<float2>("io_a32", n);
      float2* b32 = h->buf<float2>("io_b32", n);
      convert<double2, float2>(a, a32, n, h->st);
      fine_dslash<float2>(h, a32, b32, nullptr, dagger != 0, 0, nrhs, nullptr, h->st);
      convert<float2, double2>(b32, b, n, h->st);
    }
    unpack_field(h, b, reinterpret_cast<double2*>(out), nrhs);
  });
}

mgdwf_status mgdwf_set_nullvecs(mgdwf_handle h, const int32_t block[4], const double* V, int32_t nvec) {
  if (!h) return MGDWF_ERR_INVALID_ARG;
  return guarded(h, [&] {
    h->clear_graphs();
    need(block && V, MGDWF_ERR_INVALID_ARG, "null argument");
    need(h->have_gauge, MGDWF_ERR_STATE, "gauge field not set");
    (void)make_coarse(h, block, nvec);
    const long long n = h->fine_len() * nvec;
    h->V64.alloc(n * sizeof(double2));
    pack_field(h, reinterpret_cast<const double2*>(V), h->V64.as<double2>(), nvec);
    h->Vnull.alloc(n * sizeof(double2));
    MG_HIP(hipMemcpyAsync(h->Vnull.p, h->V64.p, n * sizeof(double2), hipMemcpyDeviceToDevice, h->st));
    h->nnull = nvec;
    install_basis(h, block, nvec);
  });
}

mgdwf_status mgdwf_get_nullvecs(mgdwf_handle h, double* V, int32_t* n) {
  if (!h) return MGDWF_ERR_INVALID_ARG;
  return guarded(h, [&] {
    need(n != nullptr, MGDWF_ERR_INVALID_ARG, "null count pointer");
    need(h->have_basis && h->nnull > 0, MGDWF_ERR_STATE, "no near-null vectors: run setup or set_nullvecs first");
    *n = h->nnull;
    if (!V) return;
    unpack_field(h, h->Vnull.as<double2>(), reinterpret_cast<double2*>(V), h->nnull);
    MG_HIP(hipStreamSynchronize(h->st));
  });
}

mgdwf_status mgdwf_get_basis(mgdwf_handle h, double* Vhat) {
  if (!h) return MGDWF_ERR_INVALID_ARG;
  return guarded(h, [&] {
    need(Vhat != nullptr, MGDWF_ERR_INVALID_ARG, "null output");
    need(h->have_basis, MGDWF_ERR_STATE, "no basis installed");
    unpack_field(h, h->V64.as<double2>(), reinterpret_cast<double2*>(Vhat), h->cg.Nv);
    MG_HIP(hipStreamSynchronize(h->st));
  });
}

mgdwf_status mgdwf_restrict(mgdwf_handle h, const double* fine, double* coarse, int32_t nrhs, mgdwf_prec prec) {
  if (!h) return MGDWF_ERR_INVALID_ARG;
  return guarded(h, [&] {
    need(fine && coarse && nrhs >= 1, MGDWF_ERR_INVALID_ARG, "bad argument");
    check_prec_fine(prec);
    need(h->have_basis, MGDWF_ERR_STATE, "no basis installed");
    const long long n = h->fine_len() * nrhs;
    double2* a = h->buf<double2>("io_a", n);
    pack_field(h, reinterpret_cast<const double2*>(fine), a, nrhs);
    if (prec == MGDWF_F64) {
      fine_restrict<double2>(h, h->V64.as<double2>(), a, reinterpret_cast<double2*>(coarse), nrhs);
    } else {
      const long long nc = h->coarse_len() * nrhs;
      float2* a32 = h->buf<float2>("io_a32", n);
      float2* c32 = h->buf<float2>("io_c32", nc);
      convert<double2, float2>(a, a32, n, h->st);
      fine_restrict<float2>(h, h->V32.as<float2>(), a32, c32, nrhs);
      convert<float2, double2>(c32, reinterpret_cast<double2*>(coarse), nc, h->st);
    }
  });
}
mgdwf_status mgdwf_prolong(mgdwf_handle h, const double* coarse, double* fine, int32_t nrhs, mgdwf_prec prec) {
  if (!h) return MGDWF_ERR_INVALID_ARG;
  return guarded(h, [&] {
    need(fine && coarse && nrhs >= 1, MGDWF_ERR_INVALID_ARG, "bad argument");
    check_prec_fine(prec);
    need(h->have_basis, MGDWF_ERR_STATE, "no basis installed");
    const long long n = h->fine_len() * nrhs;
    double2* a = h->buf<double2>("io_a", n);
    if (prec == MGDWF_F64) {
      fine_prolong<double2>(h, h->V64.as<double2>(), reinterpret_cast<const double2*>(coarse), a, false, nrhs);
    } else {
      const long long nc = h->coarse_len() * nrhs;
      float2* a32 = h->buf<float2>("io_a32", n);
      float2* c32 = h->buf<float2>("io_c32", nc);
      convert<double2, float2>(reinterpret_cast<const double2*>(coarse), c32, nc, h->st);
      fine_prolong<float2>(h, h->V32.as<float2>(), c32, a32, false, nrhs);
      convert<float2, double2>(a32, a, n, h->st);
    }
    unpack_field(h, a, reinterpret_cast<double2*>(fine), nrhs);
  });
}
mgdwf_status mgdwf_build_coarse(mgdwf_handle h) {
  if (!h) return MGDWF_ERR_INVALID_ARG;
  return guarded(h, [&] {
    h->clear_graphs(); build_coarse(h); });
}

mgdwf_status mgdwf_build_coarse_squared(mgdwf_handle h) {
  if (!h) return MGDWF_ERR_INVALID_ARG;
  return guarded(h, [&] {
    h->clear_graphs();
    build_coarse_squared(h);
  });
}

int32_t mgdwf_coarse_stencil_size(mgdwf_handle h) {
  if (!h || !h->have_coarse) return -1;
  return h->coarse_kind == 1 ? 33 : 9;
}

mgdwf_status mgdwf_get_coarse_op(mgdwf_handle h, double* Dc) {
  if (!h) return MGDWF_ERR_INVALID_ARG;
  return guarded(h, [&] {
    need(Dc != nullptr, MGDWF_ERR_INVALID_ARG, "null output");
    need(h->have_coarse, MGDWF_ERR_STATE, "coarse operator not built");
    if (h->coarse_kind == 1) {
      sq_canonical(h->Asq.m64.as<double2>(), reinterpret_cast<double2*>(Dc), h->cg, h->st);
      MG_HIP(hipStreamSynchronize(h->st));
      return;
    }
    long long nblk = 9LL * h->cg.Vc;
    long long tot = nblk * h->cg.n2 * h->cg.n2;
    hipLaunchKernelGGL(k_dc_canonical, dim3(ceil_div(tot, 256)), dim3(256), 0, h->st, h->Dc.m64.as<double2>(),
                       reinterpret_cast<double2*>(Dc), nblk, h->cg.n2);
    MG_LAUNCH_CHECK();
    MG_HIP(hipStreamSynchronize(h->st));
  });
}

mgdwf_status mgdwf_apply_coarse(mgdwf_handle h, const double* in, double* out, int32_t dagger, mgdwf_prec prec,
                                int32_t nrhs) {
  if (!h) return MGDWF_ERR_INVALID_ARG;
  return guarded(h, [&] {
    need(in && out && nrhs >= 1, MGDWF_ERR_INVALID_ARG, "bad argument");
    need(h->have_coarse, MGDWF_ERR_STATE, "coarse operator not built");
    need(prec >= MGDWF_F64 && prec <= MGDWF_BF16, MGDWF_ERR_INVALID_ARG, "bad coarse precision");
    const long long n = h->coarse_len() * nrhs;
    if (h->coarse_kind == 1) {  // A_c is Hermitian: the same stencil either way
      need(prec == MGDWF_F64 || prec == MGDWF_F32, MGDWF_ERR_INVALID_ARG, "the squared coarse operator is F64 or F32");
      if (prec == MGDWF_F64) {
        sq_apply64(h->Asq.m64.as<double2>(), reinterpret_cast<const double2*>(in), reinterpret_cast<double2*>(out),
                   h->cg, nrhs, h->st);
      } else {
        float2* a = h->buf<float2>("cio_a32", n);
        float2* b = h->buf<float2>("cio_b32", n);
        convert<double2, float2>(reinterpret_cast<const double2*>(in), a, n, h->st);
        sq_apply32(h->Asq.m32.as<float2>(), a, b, h->cg, nrhs, h->st);
        convert<float2, double2>(b, reinterpret_cast<double2*>(out), n, h->st);
      }
      return;
    }
    const CoarseStore& s = dagger ? h->DcH : h->Dc;
    if (prec == MGDWF_F64) {
      coarse_apply64(s, reinterpret_cast<const double2*>(in), reinterpret_cast<double2*>(out), h->cg, nrhs, h->st);
    } else {
      float2* a = h->buf<float2>("cio_a32", n);
      float2* b = h->buf<float2>("cio_b32", n);
      convert<double2, float2>(reinterpret_cast<const double2*>(in), a, n, h->st);
      coarse_apply32(s, prec, a, b, h->cg, nrhs, h->buf<char>("cio_pack", coarse_pack_bytes(h->cg, nrhs)),
                     h->g.ctile, h->st);
      convert<float2, double2>(b, reinterpret_cast<double2*>(out), n, h->st);
    }
  });
}

mgdwf_status mgdwf_apply_coarse_noalloc(mgdwf_handle h, const double* in, double* out, int32_t dagger,
                                        mgdwf_prec prec, int32_t nrhs) {
  if (!h) return MGDWF_ERR_INVALID_ARG;
  return guarded(h, [&] {
    need(in && out && nrhs >= 1, MGDWF_ERR_INVALID_ARG, "bad argument");
    need(h->have_coarse, MGDWF_ERR_STATE, "coarse operator not built");
    need(prec >= MGDWF_F64 && prec <= MGDWF_BF16, MGDWF_ERR_INVALID_ARG, "bad coarse precision");
    const bool sq = h->coarse_kind == 1;
    if (sq)
      need(prec == MGDWF_F64 || prec == MGDWF_F32, MGDWF_ERR_INVALID_ARG, "the squared coarse operator is F64 or F32");
    if (!sq && (prec == MGDWF_F16 || prec == MGDWF_BF16))
      need(h->cg.n2 % 16 == 0 && h->cg.n2 <= 64, MGDWF_ERR_INVALID_ARG,
           "16-bit coarse operator needs nvec divisible by 8 (and 2 nvec <= 64)");
    const long long n = h->coarse_len() * nrhs;
    const double2* x = reinterpret_cast<const double2*>(in);
    double2* y = reinterpret_cast<double2*>(out);
    if (prec == MGDWF_F64) {  // works on the caller's buffers directly: no scratch
      if (sq) sq_apply64(h->Asq.m64.as<double2>(), x, y, h->cg, nrhs, h->st);
      else coarse_apply64(dagger ? h->DcH : h->Dc, x, y, h->cg, nrhs, h->st);
      return;
    }
    // scratch: the FP32 input and output, then the 16-bit packed input
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t vec = up((size_t)n * sizeof(float2));
    const size_t pack = (!sq && prec != MGDWF_F32) ? coarse_pack_bytes(h->cg, nrhs) : 0;
    need(2 * vec + pack <= kScratchBytes, MGDWF_ERR_INVALID_ARG,
         "coarse vectors too large for the 16 MiB no-allocation scratch (use mgdwf_apply_coarse)");
    char* s = static_cast<char*>(h->scratch);
    float2* a = reinterpret_cast<float2*>(s);
    float2* b = reinterpret_cast<float2*>(s + vec);
    convert<double2, float2>(x, a, n, h->st);
    if (sq) sq_apply32(h->Asq.m32.as<float2>(), a, b, h->cg, nrhs, h->st);
    else coarse_apply32(dagger ? h->DcH : h->Dc, prec, a, b, h->cg, nrhs, s + 2 * vec, h->g.ctile, h->st);
    convert<float2, double2>(b, y, n, h->st);
  });
}

mgdwf_status mgdwf_setup(mgdwf_handle h, const mgdwf_mg_params* p, const double* V0, mgdwf_setup_report* report) {
  if (!h) return MGDWF_ERR_INVALID_ARG;
  return guarded(h, [&] {
    h->clear_graphs();
    check_params(h, p);
    need(V0 != nullptr, MGDWF_ERR_INVALID_ARG, "null starting vectors");
    need(h->have_gauge, MGDWF_ERR_STATE, "gauge field not set");
    if (report) std::memset(report, 0, sizeof(*report));
    const int nh = p->squared ? p->nvec : p->nvec / 2;
    double2* W = h->buf<double2>("setup_w", h->fine_len() * nh);
    pack_field(h, reinterpret_cast<const double2*>(V0), W, nh);
    mg_setup(h, *p, W, report);
  });
}

mgdwf_status mgdwf_set_mg_params(mgdwf_handle h, const mgdwf_mg_params* p) {
  if (!h) return MGDWF_ERR_INVALID_ARG;
  return guarded(h, [&] {
    h->clear_graphs();
    check_params(h, p);
    need(h->have_coarse, MGDWF_ERR_STATE, "no basis / coarse operator installed");
    need(p->nvec == h->cg.Nv, MGDWF_ERR_INVALID_ARG, "nvec differs from the installed basis");
    need(p->squared == h->coarse_kind, MGDWF_ERR_STATE,
         p->squared ? "squared = 1 needs mgdwf_build_coarse_squared (or a squared setup) first"
                    : "squared = 0 needs the 9-point operator (mgdwf_build_coarse) first");
    for (int m = 0; m < 4; ++m) need(p->block[m] == h->cg.block[m], MGDWF_ERR_INVALID_ARG, "block differs from the installed basis");
    h->mp = *p;
    h->have_params = true;
  });
}

mgdwf_status mgdwf_solve(mgdwf_handle h, const double* b, double* x, int32_t nrhs, const mgdwf_solve_params* p,
                         mgdwf_solve_report* reports) {
  if (!h) return MGDWF_ERR_INVALID_ARG;
  double2* x64 = nullptr;
  mgdwf_status st = guarded(h, [&] {
    need(b && x && p && nrhs >= 1, MGDWF_ERR_INVALID_ARG, "bad argument");
    need(p->tol > 0 && p->max_outer >= 1 && p->restart >= 1, MGDWF_ERR_INVALID_ARG, "bad solve parameters");
    need(h->have_coarse && h->have_params, MGDWF_ERR_STATE, "setup (or set_nullvecs + build_coarse + set_mg_params) first");
    const long long n = h->fine_len() * nrhs;
    double2* b64 = h->buf<double2>("sol_b", n);
    x64 = h->buf<double2>("sol_x", n);
    pack_field(h, reinterpret_cast<const double2*>(b), b64, nrhs);
    pack_field(h, reinterpret_cast<const double2*>(x), x64, nrhs);
    mg_solve(h, b64, x64, nrhs, *p, reports);
  });
  if ((st == MGDWF_OK || st == MGDWF_ERR_NOT_CONVERGED) && x64) {
    mgdwf_status s2 = guarded(h, [&] {
      unpack_field(h, x64, reinterpret_cast<double2*>(x), nrhs);
      MG_HIP(hipStreamSynchronize(h->st));
    });
    if (s2 != MGDWF_OK) return s2;
  }
  return st;
}

mgdwf_status mgdwf_apply_vcycle(mgdwf_handle h, const double* in, double* out, int32_t nrhs) {
  if (!h) return MGDWF_ERR_INVALID_ARG;
  return guarded(h, [&] {
    need(in && out && nrhs >= 1, MGDWF_ERR_INVALID_ARG, "bad argument");
    need(h->have_coarse && h->have_params, MGDWF_ERR_STATE, "setup (or set_nullvecs + build_coarse + set_mg_params) first");
    const long long n = h->fine_len() * nrhs;
    double2* a = h->buf<double2>("io_a", n);
    double2* b = h->buf<double2>("io_b", n);
    pack_field(h, reinterpret_cast<const double2*>(in), a, nrhs);
    vcycle_apply(h, a, b, nrhs);
    unpack_field(h, b, reinterpret_cast<double2*>(out), nrhs);
    MG_HIP(hipStreamSynchronize(h->st));
  });
}

mgdwf_status mgdwf_low_modes(mgdwf_handle h, const double* v0, int32_t nev, int32_t m, double solve_tol,
                             double* evals, double* evecs, double* resid) {
  if (!h) return MGDWF_ERR_INVALID_ARG;
  return guarded(h, [&] {
    need(v0 && evals, MGDWF_ERR_INVALID_ARG, "null argument");
    need_4d(h, "mgdwf_low_modes");
    need(nev >= 1 && m >= nev && m <= 256, MGDWF_ERR_INVALID_ARG, "need 1 <= nev <= m <= 256");
    need(solve_tol > 0.0 && solve_tol <= 1e-3, MGDWF_ERR_INVALID_ARG, "solve_tol must be in (0, 1e-3]");
    need(h->have_coarse && h->have_params, MGDWF_ERR_STATE, "the Lanczos steps solve with the multigrid: set it up first");
    const long long nf = h->fine_len();
    double2* a = h->buf<double2>("io_a", nf);
    pack_fermion_f64(reinterpret_cast<const double2*>(v0), a, h->g, 1, h->st);
    double2* ev = evecs ? h->buf<double2>("lm_evecs", (size_t)nev * nf) : nullptr;
    low_modes(h, a, nev, m, solve_tol, evals, ev, resid);
    if (evecs) unpack_fermion_f64(ev, reinterpret_cast<double2*>(evecs), h->g, nev, h->st);
    MG_HIP(hipStreamSynchronize(h->st));
    for (auto it = h->ws.begin(); it != h->ws.end();)  // the Krylov basis is large: give it back
      it = it->first.rfind("lm_", 0) == 0 ? h->ws.erase(it) : std::next(it);
    ++h->ws_gen;  // captured graphs keyed on the old workspaces are not replayed
  });
}

mgdwf_status mgdwf_coarse_coverage(mgdwf_handle h, const double* e, int32_t n, double* frac) {
  if (!h) return MGDWF_ERR_INVALID_ARG;
  return guarded(h, [&] {
    need(e && frac && n >= 1, MGDWF_ERR_INVALID_ARG, "bad argument");
    need(h->have_basis, MGDWF_ERR_STATE, "no basis installed");
    double2* a = h->buf<double2>("io_a", h->fine_len() * n);
    pack_field(h, reinterpret_cast<const double2*>(e), a, n);
    coarse_coverage(h, a, n, frac);
  });
}

mgdwf_status mgdwf_setup_level2(mgdwf_handle h, const mgdwf_level2_params* p, const double* W0,
                                double* null_residual) {
  if (!h) return MGDWF_ERR_INVALID_ARG;
  return guarded(h, [&] {
    need(p && W0, MGDWF_ERR_INVALID_ARG, "null argument");
    setup_level2(h, *p, reinterpret_cast<const double2*>(W0), null_residual);
  });
}

mgdwf_status mgdwf_set_level2_params(mgdwf_handle h, const mgdwf_level2_params* p) {
  if (!h) return MGDWF_ERR_INVALID_ARG;
  return guarded(h, [&] {
    need(p != nullptr, MGDWF_ERR_INVALID_ARG, "null argument");
    need(h->have_l2, MGDWF_ERR_STATE, "no third level installed");
    for (int m = 0; m < 4; ++m)
      need(p->block[m] == h->l2p.block[m], MGDWF_ERR_INVALID_ARG, "level-2 block differs from the installed one");
    need(p->nvec == h->l2p.nvec, MGDWF_ERR_INVALID_ARG, "level-2 nvec differs from the installed one");
    need(p->nu >= 0 && p->coarse_maxiter >= 1 && p->gamma >= 0 && p->gamma <= 4 && p->coarse_tol >= 0.0,
         MGDWF_ERR_INVALID_ARG, "bad level-2 parameters");
    h->clear_graphs();
    h->l2p = *p;
  });
}

mgdwf_status mgdwf_get_level2(mgdwf_handle h, double* W, double* What, double* Acc) {
  if (!h) return MGDWF_ERR_INVALID_ARG;
  return guarded(h, [&] {
    need(h->have_l2, MGDWF_ERR_STATE, "no third level installed");
    const size_t nb = (size_t)h->l2p.nvec * h->coarse_len() * sizeof(double2);
    if (W) MG_HIP(hipMemcpyAsync(W, h->W2null.p, nb, hipMemcpyDeviceToDevice, h->st));
    if (What) MG_HIP(hipMemcpyAsync(What, h->W2_64.p, nb, hipMemcpyDeviceToDevice, h->st));
    if (Acc) sq_canonical(h->Acc64.as<double2>(), reinterpret_cast<double2*>(Acc), h->cg2, h->st);
    MG_HIP(hipStreamSynchronize(h->st));
  });
}

// ---------------------------------------------------------------- setup checkpoints
namespace {

constexpr char kCkMagic[8] = {'M', 'G', 'D', 'W', 'F', 'C', 'K', '1'};

struct CkHeader {
  char magic[8];
  int32_t L[4], Ls, bc[4], block[4], nvec, nnull, coarse_kind, pad;
  double M5, mf;
  uint64_t gauge_checksum;
  int64_t fine_len;
};

// FNV-1a over the bytes of the installed FP64 links (internal layout)
uint64_t gauge_checksum(mgdwf_ctx* h) {
  std::vector<unsigned char> host(h->U64.bytes);
  MG_HIP(hipMemcpyAsync(host.data(), h->U64.p, host.size(), hipMemcpyDeviceToHost, h->st));
  MG_HIP(hipStreamSynchronize(h->st));
  uint64_t x = 1469598103934665603ULL;
  for (unsigned char c : host) {
    x ^= c;
    x *= 1099511628211ULL;
  }
  return x;
}

struct File {
  FILE* f = nullptr;
  ~File() { if (f) fclose(f); }
};

// n fields of the internal FP64 layout, written or read as canonical complex128
void write_fields(mgdwf_ctx* h, FILE* f, const double2* dev, int n) {
  const long long nf = h->fine_len();
  double2* canon = h->buf<double2>("ck_canon", nf);
  std::vector<double2> host(nf);
  for (int k = 0; k < n; ++k) {
    unpack_field(h, dev + k * nf, canon, 1);
    MG_HIP(hipMemcpyAsync(host.data(), canon, nf * sizeof(double2), hipMemcpyDeviceToHost, h->st));
    MG_HIP(hipStreamSynchronize(h->st));
    need(fwrite(host.data(), sizeof(double2), nf, f) == (size_t)nf, MGDWF_ERR_INVALID_ARG, "checkpoint write failed");
  }
}

void read_fields(mgdwf_ctx* h, FILE* f, double2* dev, int n) {
  const long long nf = h->fine_len();
  double2* canon = h->buf<double2>("ck_canon", nf);
  std::vector<double2> host(nf);
  for (int k = 0; k < n; ++k) {
    need(fread(host.data(), sizeof(double2), nf, f) == (size_t)nf, MGDWF_ERR_INVALID_ARG, "checkpoint is truncated");
    MG_HIP(hipMemcpyAsync(canon, host.data(), nf * sizeof(double2), hipMemcpyHostToDevice, h->st));
    pack_field(h, canon, dev + k * nf, 1);
    MG_HIP(hipStreamSynchronize(h->st));
  }
}

}  // namespace

mgdwf_status mgdwf_save_setup(mgdwf_handle h, const char* path) {
  if (!h) return MGDWF_ERR_INVALID_ARG;
  return guarded(h, [&] {
    need(path != nullptr, MGDWF_ERR_INVALID_ARG, "null path");
    need(h->have_gauge && h->have_basis && h->have_coarse, MGDWF_ERR_STATE,
         "nothing to save: set the gauge field and run a setup first");
    CkHeader hd{};
    std::memcpy(hd.magic, kCkMagic, 8);
    for (int m = 0; m < 4; ++m) {
      hd.L[m] = h->g.L[m];
      hd.bc[m] = h->g.bc[m];
      hd.block[m] = h->cg.block[m];
    }
    hd.Ls = h->g.Ls;
    hd.nvec = h->cg.Nv;
    hd.nnull = h->nnull;
    hd.coarse_kind = h->coarse_kind;
    hd.M5 = h->M5;
    hd.mf = h->mf;
    hd.gauge_checksum = gauge_checksum(h);
    hd.fine_len = h->fine_len();
    File fh;
    fh.f = fopen(path, "wb");
    need(fh.f != nullptr, MGDWF_ERR_INVALID_ARG, (std::string("cannot open ") + path + " for writing").c_str());
    need(fwrite(&hd, sizeof hd, 1, fh.f) == 1, MGDWF_ERR_INVALID_ARG, "checkpoint write failed");
    write_fields(h, fh.f, h->V64.as<double2>(), hd.nvec);
    if (hd.nnull > 0) write_fields(h, fh.f, h->Vnull.as<double2>(), hd.nnull);
    need(fflush(fh.f) == 0, MGDWF_ERR_INVALID_ARG, "checkpoint write failed");
    h->ws.erase("ck_canon");
    ++h->ws_gen;
  });
}

mgdwf_status mgdwf_load_setup(mgdwf_handle h, const char* path) {
  if (!h) return MGDWF_ERR_INVALID_ARG;
  return guarded(h, [&] {
    need(path != nullptr, MGDWF_ERR_INVALID_ARG, "null path");
    need(h->have_gauge, MGDWF_ERR_STATE, "gauge field not set");
    File fh;
    fh.f = fopen(path, "rb");
    need(fh.f != nullptr, MGDWF_ERR_INVALID_ARG, (std::string("cannot open ") + path).c_str());
    CkHeader hd{};
    need(fread(&hd, sizeof hd, 1, fh.f) == 1 && std::memcmp(hd.magic, kCkMagic, 8) == 0, MGDWF_ERR_INVALID_ARG,
         "not a setup checkpoint");
    bool same = hd.Ls == h->g.Ls && hd.M5 == h->M5 && hd.mf == h->mf && hd.fine_len == h->fine_len();
    for (int m = 0; m < 4; ++m) same = same && hd.L[m] == h->g.L[m] && hd.bc[m] == h->g.bc[m];
    need(same, MGDWF_ERR_STATE, "the checkpoint was taken on another lattice or action");
    need(hd.gauge_checksum == gauge_checksum(h), MGDWF_ERR_STATE, "the checkpoint was taken on another gauge field");
    need(hd.nvec >= 1 && hd.nnull >= 0 && (hd.coarse_kind == 0 || hd.coarse_kind == 1), MGDWF_ERR_INVALID_ARG,
         "corrupt checkpoint header");
    h->clear_graphs();
    h->have_basis = h->have_coarse = h->have_params = false;
    const CoarseGeometry cg = make_coarse(h, hd.block, hd.nvec);
    const long long nf = h->fine_len();
    h->V64.alloc((size_t)hd.nvec * nf * sizeof(double2));
    read_fields(h, fh.f, h->V64.as<double2>(), hd.nvec);
    if (hd.nnull > 0) {
      h->Vnull.alloc((size_t)hd.nnull * nf * sizeof(double2));
      read_fields(h, fh.f, h->Vnull.as<double2>(), hd.nnull);
    }
    h->nnull = hd.nnull;
    // the basis as saved (already orthonormal: installed as is, so the
    // coarse operator and every later solve repeat the saved handle's bitwise)
    h->cg = cg;
    h->V32.alloc((size_t)hd.nvec * nf * sizeof(float2));
    convert<double2, float2>(h->V64.as<double2>(), h->V32.as<float2>(), (long long)hd.nvec * nf, h->st);
    MG_HIP(hipStreamSynchronize(h->st));
    h->have_basis = true;
    if (hd.coarse_kind == 1) build_coarse_squared(h);
    else build_coarse(h);
    h->ws.erase("ck_canon");
    ++h->ws_gen;
  });
}

mgdwf_status mgdwf_trim(mgdwf_handle h) {
  if (!h) return MGDWF_ERR_INVALID_ARG;
  return guarded(h, [&] {
    MG_HIP(hipStreamSynchronize(h->st));
    h->clear_graphs();
    h->ws.clear();
    h->ptr_cache.clear();
  });
}

int64_t mgdwf_memory_bytes(mgdwf_handle h) {
  if (!h) return -1;
  long long n = (long long)(h->U64.bytes + h->U32.bytes + h->V64.bytes + h->V32.bytes);
  for (const mgdwf::CoarseStore* cs : {&h->Dc, &h->DcH, &h->Asq})
    n += (long long)(cs->m64.bytes + cs->m32.bytes + cs->re16.bytes + cs->im16.bytes + cs->sc16.bytes +
                     cs->reb.bytes + cs->imb.bytes + cs->scb.bytes);
  for (const auto& kv : h->ws) n += (long long)kv.second.bytes;
  return n;
}

mgdwf_status mgdwf_solve_batch(const mgdwf_handle* hs, int32_t n, const double* const* b, double* const* x,
                               const int32_t* nrhs, const mgdwf_solve_params* p, mgdwf_solve_report* reports) {
  if (!hs || !b || !x || !nrhs || !p || !reports || n < 1) return MGDWF_ERR_INVALID_ARG;
  for (int i = 0; i < n; ++i) {
    if (!hs[i] || nrhs[i] < 1) return MGDWF_ERR_INVALID_ARG;
    for (int j = 0; j < i; ++j)
      if (hs[j] == hs[i]) return MGDWF_ERR_INVALID_ARG;  // a handle is not thread-safe
  }
  std::vector<mgdwf_status> st((size_t)n, MGDWF_OK);
  std::vector<long long> off((size_t)n, 0);
  for (int i = 1; i < n; ++i) off[i] = off[i - 1] + nrhs[i - 1];
  std::vector<std::thread> th;
  th.reserve((size_t)n);
  for (int i = 0; i < n; ++i)
    th.emplace_back([&, i] {
      if (hipSetDevice(hs[i]->device) != hipSuccess) {
        st[i] = MGDWF_ERR_HIP;
        hs[i]->err = "hipSetDevice failed";
        return;
      }
      st[i] = mgdwf_solve(hs[i], b[i], x[i], nrhs[i], p, reports + off[i]);
    });
  for (auto& t : th) t.join();
  mgdwf_status worst = MGDWF_OK;
  for (int i = 0; i < n; ++i)
    if (st[i] != MGDWF_OK && (worst == MGDWF_OK || worst == MGDWF_ERR_NOT_CONVERGED)) worst = st[i];
  return worst;
}

mgdwf_status mgdwf_cgne(mgdwf_handle h, const double* b, double* x, const mgdwf_solve_params* p,
                        mgdwf_solve_report* report) {
  if (!h) return MGDWF_ERR_INVALID_ARG;
  double2* x64 = nullptr;
  mgdwf_status st = guarded(h, [&] {
    need(b && x && p, MGDWF_ERR_INVALID_ARG, "bad argument");
    need(p->tol > 0 && p->max_outer >= 1, MGDWF_ERR_INVALID_ARG, "bad solve parameters");
    need(h->have_gauge, MGDWF_ERR_STATE, "gauge field not set");
    const long long n = h->fine_len();
    double2* b64 = h->buf<double2>("sol_b", n);
    x64 = h->buf<double2>("sol_x", n);
    pack_field(h, reinterpret_cast<const double2*>(b), b64, 1);
    pack_field(h, reinterpret_cast<const double2*>(x), x64, 1);
    cgne_solve(h, b64, x64, *p, report);
  });
  if ((st == MGDWF_OK || st == MGDWF_ERR_NOT_CONVERGED) && x64) {
    mgdwf_status s2 = guarded(h, [&] {
      unpack_field(h, x64, reinterpret_cast<double2*>(x), 1);
      MG_HIP(hipStreamSynchronize(h->st));
    });
    if (s2 != MGDWF_OK) return s2;
  }
  return st;
}

mgdwf_status mgdwf_time_kernel(mgdwf_handle h, mgdwf_kernel k, mgdwf_prec prec, int32_t nrhs, int32_t iters, double* ms) {
  if (!h) return MGDWF_ERR_INVALID_ARG;
  return guarded(h, [&] {
    need(ms && iters >= 1 && nrhs >= 1, MGDWF_ERR_INVALID_ARG, "bad argument");
    if (k == MGDWF_K_COARSE)
      need(prec >= MGDWF_F64 && prec <= MGDWF_BF16, MGDWF_ERR_INVALID_ARG, "bad coarse precision");
    else
      check_prec_fine(prec);
    need(h->have_gauge, MGDWF_ERR_STATE, "gauge field not set");
    const long long nf = h->fine_len() * nrhs;
    hipEvent_t e0, e1;
    MG_HIP(hipEventCreate(&e0));
    MG_HIP(hipEventCreate(&e1));
    auto run = [&](int reps) {
      for (int i = 0; i < reps; ++i) {
        if (k == MGDWF_K_DSLASH) {
          if (prec == MGDWF_F64)
            fine_dslash<double2>(h, h->buf<double2>("t_a", nf), h->buf<double2>("t_b", nf), nullptr, false, 0, nrhs,
                                 nullptr, h->st);
          else
            fine_dslash<float2>(h, h->buf<float2>("t_a32", nf), h->buf<float2>("t_b32", nf), nullptr, false, 0, nrhs,
                                nullptr, h->st);
        } else {
          need(h->have_coarse, MGDWF_ERR_STATE, "coarse operator not built");
          const long long nc = h->coarse_len() * nrhs;
          if (k == MGDWF_K_RESTRICT) {
            if (prec == MGDWF_F64)
              fine_restrict<double2>(h, h->V64.as<double2>(), h->buf<double2>("t_a", nf), h->buf<double2>("t_c", nc),
                                     nrhs);
            else
              fine_restrict<float2>(h, h->V32.as<float2>(), h->buf<float2>("t_a32", nf), h->buf<float2>("t_c32", nc),
                                    nrhs);
          } else if (k == MGDWF_K_PROLONG) {
            if (prec == MGDWF_F64)
              fine_prolong<double2>(h, h->V64.as<double2>(), h->buf<double2>("t_c", nc), h->buf<double2>("t_a", nf),
                                    false, nrhs);
            else
              fine_prolong<float2>(h, h->V32.as<float2>(), h->buf<float2>("t_c32", nc), h->buf<float2>("t_a32", nf),
                                   false, nrhs);
          } else if (k == MGDWF_K_COARSE && h->coarse_kind == 1) {
            need(prec == MGDWF_F64 || prec == MGDWF_F32, MGDWF_ERR_INVALID_ARG, "the squared coarse operator is F64 or F32");
            if (prec == MGDWF_F64)
              sq_apply64(h->Asq.m64.as<double2>(), h->buf<double2>("t_c", nc), h->buf<double2>("t_d", nc), h->cg, nrhs,
                         h->st);
            else
              sq_apply32(h->Asq.m32.as<float2>(), h->buf<float2>("t_c32", nc), h->buf<float2>("t_d32", nc), h->cg,
                         nrhs, h->st);
          } else if (k == MGDWF_K_COARSE) {
            if (prec == MGDWF_F64)
              coarse_apply64(h->Dc, h->buf<double2>("t_c", nc), h->buf<double2>("t_d", nc), h->cg, nrhs, h->st);
            else
              coarse_apply32(h->Dc, prec, h->buf<float2>("t_c32", nc), h->buf<float2>("t_d32", nc), h->cg, nrhs,
                             h->buf<char>("t_pack", coarse_pack_bytes(h->cg, nrhs)), h->g.ctile, h->st);
          } else {
            fail(MGDWF_ERR_INVALID_ARG, "unknown kernel id");
          }
        }
      }
    };
    // fill the inputs once so the timed kernels read finite data
    {
      if (k == MGDWF_K_DSLASH || k == MGDWF_K_RESTRICT) {
        if (prec == MGDWF_F64) zero<double2>(h->buf<double2>("t_a", nf), nf, h->st);
        else zero<float2>(h->buf<float2>("t_a32", nf), nf, h->st);
      } else {
        const long long nc = h->coarse_len() * nrhs;
        if (prec == MGDWF_F64) zero<double2>(h->buf<double2>("t_c", nc), nc, h->st);
        else zero<float2>(h->buf<float2>("t_c32", nc), nc, h->st);
      }
    }
    run(2);  // warm-up
    MG_HIP(hipEventRecord(e0, h->st));
    run(iters);
    MG_HIP(hipEventRecord(e1, h->st));
    MG_HIP(hipEventSynchronize(e1));
    float t = 0.f;
    MG_HIP(hipEventElapsedTime(&t, e0, e1));
    *ms = (double)t / iters;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  });
}

mgdwf_status mgdwf_tune(mgdwf_handle h, int32_t nrhs, int32_t iters, mgdwf_tune_report* rep) {
  if (!h) return MGDWF_ERR_INVALID_ARG;
  return guarded(h, [&] {
    need(rep && iters >= 1 && nrhs >= 1, MGDWF_ERR_INVALID_ARG, "bad argument");
    need_4d(h, "mgdwf_tune");
    need(h->have_gauge, MGDWF_ERR_STATE, "gauge field not set");
    std::memset(rep, 0, sizeof(*rep));
    rep->chosen = -1;
    const long long nf = h->fine_len() * nrhs;
    float2* a = h->buf<float2>("t_a32", nf);
    float2* b = h->buf<float2>("t_b32", nf);
    zero<float2>(a, nf, h->st);
    struct Events {
      hipEvent_t e0 = nullptr, e1 = nullptr;
      ~Events() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
      }
    } ev;
    MG_HIP(hipEventCreate(&ev.e0));
    MG_HIP(hipEventCreate(&ev.e1));
    int best = -1, dflt = -1, dflt_j = -1;
    double best_us = 0.0, dflt_us = 0.0;
    for (int i = 0; i < dslash_ftile_count() && rep->ntilings < MGDWF_MAX_TILINGS; ++i) {
      Geometry g = h->g;
      g.ftile = i;
      int desc[4], flags = 0;
      if (!dslash_ftile_desc(g, i, nrhs, desc, &flags)) continue;
      auto run = [&](int n) {
        for (int k = 0; k < n; ++k)
          dslash_ex<float2>(a, b, nullptr, h->U32.as<float2>(), g, h->M5, h->mf, (k & 1) != 0, 0, nrhs, nullptr,
                            h->st);
      };
      run(2);
      MG_HIP(hipEventRecord(ev.e0, h->st));
      run(iters);
      MG_HIP(hipEventRecord(ev.e1, h->st));
      MG_HIP(hipEventSynchronize(ev.e1));
      float ms = 0.f;
      MG_HIP(hipEventElapsedTime(&ms, ev.e0, ev.e1));
      const double us = 1e3 * ms / iters;
      const int j = rep->ntilings++;
      rep->id[j] = i;
      rep->flags[j] = flags;
      for (int q = 0; q < 4; ++q) rep->tile[j][q] = desc[q];
      rep->us[j] = us;
      if (dflt < 0) {
        dflt = i;
        dflt_j = j;
        dflt_us = us;
      }
      if (best < 0 || us < best_us) {
        best = i;
        best_us = us;
        rep->chosen = j;
      }
    }
    if (best >= 0 && best_us > 0.97 * dflt_us) {  // within noise of the default: keep it
      best = dflt;
      rep->chosen = dflt_j;
    }
    if (best >= 0) h->g.ftile = best;
    h->clear_graphs();  // captured launches carry the old tiling
    // MFMA shape of the 16-bit coarse apply, timed on the FP16 store (the BF16
    // one has the same shape), when a coarse operator is built
    rep->coarse_chosen = -1;
    if (h->have_coarse && h->cg.n2 % 16 == 0) {
      const long long nc = h->coarse_len() * nrhs;
      float2* ca = h->buf<float2>("t_c32", nc);
      float2* cb = h->buf<float2>("t_d32", nc);
      zero<float2>(ca, nc, h->st);
      char* pk = h->buf<char>("t_pack", coarse_pack_bytes(h->cg, nrhs));
      for (int ct = 0; ct < 2; ++ct) {
        auto run = [&](int n) {
          for (int k = 0; k < n; ++k) coarse_apply32(h->Dc, MGDWF_F16, ca, cb, h->cg, nrhs, pk, ct, h->st);
        };
        run(2);
        MG_HIP(hipEventRecord(ev.e0, h->st));
        run(4 * iters);
        MG_HIP(hipEventRecord(ev.e1, h->st));
        MG_HIP(hipEventSynchronize(ev.e1));
        float ms = 0.f;
        MG_HIP(hipEventElapsedTime(&ms, ev.e0, ev.e1));
        rep->coarse_us[ct] = 1e3 * ms / (4 * iters);
      }
      rep->coarse_chosen = rep->coarse_us[1] <= 0.97 * rep->coarse_us[0] ? 1 : 0;
      h->g.ctile = rep->coarse_chosen;
    }
  });
}

mgdwf_status mgdwf_set_barrier_timeout(mgdwf_handle h, double seconds) {
  if (!h) return MGDWF_ERR_INVALID_ARG;
  return guarded(h, [&] {
    need(std::isfinite(seconds) && seconds >= 0.0 && seconds <= 3600.0, MGDWF_ERR_INVALID_ARG,
         "timeout must be in [0, 3600] seconds");
    h->barrier_wait_s = seconds;
  });
}

mgdwf_status mgdwf_set_coarse_tiling(mgdwf_handle h, int32_t id) {
  if (!h) return MGDWF_ERR_INVALID_ARG;
  return guarded(h, [&] {
    need(id >= -1 && id <= 1, MGDWF_ERR_INVALID_ARG, "coarse tiling id must be -1, 0 or 1");
    h->g.ctile = id < 0 ? 0 : id;
    h->clear_graphs();
  });
}

mgdwf_status mgdwf_set_tiling(mgdwf_handle h, int32_t id) {
  if (!h) return MGDWF_ERR_INVALID_ARG;
  return guarded(h, [&] {
    int desc[4], flags = 0;
    need_4d(h, "mgdwf_set_tiling");
    need(id == -1 || dslash_ftile_desc(h->g, id, 1, desc, &flags), MGDWF_ERR_INVALID_ARG,
         "tiling does not apply to this lattice");
    h->g.ftile = id;
    h->clear_graphs();
  });
}

}  // extern "C"

// ---------------------------------------------------------------- learned proposals
#include "nullnet.h"

struct mgdwf_net_s {
  mgdwf::NullNet net;
  std::string err;
};

namespace {
template <class F>
mgdwf_status guarded_net(mgdwf_net n, mgdwf_handle h, F&& f) {
  try {
    if (h) need_4d(h, "the near-null proposal network");
    f();
    return MGDWF_OK;
  } catch (const Error& e) {
    if (h) h->err = e.msg;
    if (n) n->err = e.msg;
    if (!h && !n) g_create_error = e.msg;
    return e.code;
  } catch (const std::exception& e) {
    if (h) h->err = e.what();
    if (n) n->err = e.what();
    return MGDWF_ERR_HIP;
  }
}
}  // namespace

extern "C" {

mgdwf_status mgdwf_net_create(const mgdwf_net_config* cfg, mgdwf_net* out) {
  return guarded_net(nullptr, nullptr, [&] {
    need(cfg && out, MGDWF_ERR_INVALID_ARG, "null argument");
    for (int l = 0; l < 5; ++l) need(cfg->channels[l] >= 1 && cfg->channels[l] <= 64, MGDWF_ERR_INVALID_ARG, "channels must be in 1..64");
    need(cfg->channels[4] % 4 == 0, MGDWF_ERR_INVALID_ARG, "output channels must be 4 x proposals");
    need(cfg->lam >= 0.0, MGDWF_ERR_INVALID_ARG, "lam must be >= 0");
    auto* n = new mgdwf_net_s();
    for (int l = 0; l < 5; ++l) n->net.ch[l] = cfg->channels[l];
    n->net.lam = cfg->lam;
    try {
      n->net.init(cfg->seed);
    } catch (...) {
      delete n;
      throw;
    }
    *out = n;
  });
}

mgdwf_status mgdwf_net_destroy(mgdwf_net net) {
  delete net;
  return MGDWF_OK;
}

int64_t mgdwf_net_num_weights(mgdwf_net net) { return net ? net->net.nweights() : 0; }

const char* mgdwf_net_last_error(mgdwf_net net) { return net ? net->err.c_str() : g_create_error.c_str(); }

mgdwf_status mgdwf_net_set_weights(mgdwf_net net, const float* w) {
  if (!net) return MGDWF_ERR_INVALID_ARG;
  return guarded_net(net, nullptr, [&] {
    need(w != nullptr, MGDWF_ERR_INVALID_ARG, "null weights");
    net->net.set_weights(w, nullptr);
  });
}

mgdwf_status mgdwf_net_get_weights(mgdwf_net net, float* w) {
  if (!net) return MGDWF_ERR_INVALID_ARG;
  return guarded_net(net, nullptr, [&] {
    need(w != nullptr, MGDWF_ERR_INVALID_ARG, "null output");
    MG_HIP(hipMemcpy(w, net->net.w.p, net->net.nweights() * sizeof(float), hipMemcpyDeviceToHost));
  });
}

mgdwf_status mgdwf_net_propose(mgdwf_net net, mgdwf_handle h, const double* eta, double* V) {
  if (!net || !h) return MGDWF_ERR_INVALID_ARG;
  return guarded_net(net, h, [&] {
    need(eta && V, MGDWF_ERR_INVALID_ARG, "null argument");
    need(h->have_gauge, MGDWF_ERR_STATE, "gauge field not set");
    mgdwf::net_propose(net->net, h, reinterpret_cast<const double2*>(eta), reinterpret_cast<double2*>(V));
  });
}

mgdwf_status mgdwf_net_grad(mgdwf_net net, mgdwf_handle h, const double* eta, double* loss, float* grad) {
  if (!net || !h) return MGDWF_ERR_INVALID_ARG;
  return guarded_net(net, h, [&] {
    need(eta && loss, MGDWF_ERR_INVALID_ARG, "null argument");
    need(h->have_gauge, MGDWF_ERR_STATE, "gauge field not set");
    *loss = mgdwf::net_grad(net->net, h, reinterpret_cast<const double2*>(eta));
    if (grad) MG_HIP(hipMemcpy(grad, net->net.g.p, net->net.nweights() * sizeof(float), hipMemcpyDeviceToHost));
  });
}

mgdwf_status mgdwf_net_train_step(mgdwf_net net, mgdwf_handle h, const double* eta, double lr, double* loss) {
  if (!net || !h) return MGDWF_ERR_INVALID_ARG;
  return guarded_net(net, h, [&] {
    need(eta && loss && lr > 0, MGDWF_ERR_INVALID_ARG, "bad argument");
    need(h->have_gauge, MGDWF_ERR_STATE, "gauge field not set");
    *loss = mgdwf::net_train_step(net->net, h, reinterpret_cast<const double2*>(eta), lr);
  });
}

mgdwf_status mgdwf_net_train(mgdwf_net net, const mgdwf_handle* hs, int32_t n, const double* const* etas,
                             int32_t steps, double lr, double lr_final, double* losses) {
  if (!net || !hs || !etas || n < 1 || steps < 1) return MGDWF_ERR_INVALID_ARG;
  for (int i = 0; i < n; ++i)
    if (!hs[i]) return MGDWF_ERR_INVALID_ARG;
  return guarded_net(net, nullptr, [&] {
    need(lr > 0 && lr_final > 0, MGDWF_ERR_INVALID_ARG, "learning rates must be > 0");
    for (int i = 0; i < n; ++i) {
      need_4d(hs[i], "the near-null proposal network");
      need(hs[i]->have_gauge && hs[i]->have_basis, MGDWF_ERR_STATE, "every handle needs its gauge field and target basis");
    }
    for (int k = 0; k < steps; ++k) {
      need(etas[k] != nullptr, MGDWF_ERR_INVALID_ARG, "null input draw");
      mgdwf_handle h = hs[k % n];
      const double a = lr * std::pow(lr_final / lr, (double)k / std::max(1, steps - 1));
      const double l = mgdwf::net_train_step(net->net, h, reinterpret_cast<const double2*>(etas[k]), a);
      if (losses) losses[k] = l;
    }
  });
}

// ---- network files: magic, int32 channels[5], double lam, int64 Adam step,
// int64 weight count, then FP32 master weights and the two Adam moments
namespace {
constexpr char kNetMagic[8] = {'M', 'G', 'D', 'W', 'F', 'N', 'N', '1'};
}

mgdwf_status mgdwf_net_save(mgdwf_net net, const char* path) {
  if (!net) return MGDWF_ERR_INVALID_ARG;
  return guarded_net(net, nullptr, [&] {
    need(path != nullptr, MGDWF_ERR_INVALID_ARG, "null path");
    const long long nw = net->net.nweights();
    std::vector<float> host(3 * nw);
    MG_HIP(hipMemcpy(host.data(), net->net.w.p, nw * sizeof(float), hipMemcpyDeviceToHost));
    MG_HIP(hipMemcpy(host.data() + nw, net->net.m.p, nw * sizeof(float), hipMemcpyDeviceToHost));
    MG_HIP(hipMemcpy(host.data() + 2 * nw, net->net.v.p, nw * sizeof(float), hipMemcpyDeviceToHost));
    FILE* f = std::fopen(path, "wb");
    need(f != nullptr, MGDWF_ERR_INVALID_ARG, "cannot open the network file for writing");
    int32_t ch[5];
    for (int l = 0; l < 5; ++l) ch[l] = net->net.ch[l];
    const int64_t step = net->net.step, n64 = nw;
    bool ok = std::fwrite(kNetMagic, 1, 8, f) == 8 && std::fwrite(ch, sizeof ch, 1, f) == 1 &&
              std::fwrite(&net->net.lam, sizeof(double), 1, f) == 1 && std::fwrite(&step, 8, 1, f) == 1 &&
              std::fwrite(&n64, 8, 1, f) == 1 &&
              std::fwrite(host.data(), sizeof(float), host.size(), f) == host.size();
    ok = (std::fclose(f) == 0) && ok;
    need(ok, MGDWF_ERR_INVALID_ARG, "writing the network file failed");
  });
}

mgdwf_status mgdwf_net_load(mgdwf_net net, const char* path) {
  if (!net) return MGDWF_ERR_INVALID_ARG;
  return guarded_net(net, nullptr, [&] {
    need(path != nullptr, MGDWF_ERR_INVALID_ARG, "null path");
    FILE* f = std::fopen(path, "rb");
    need(f != nullptr, MGDWF_ERR_INVALID_ARG, "cannot open the network file");
    char magic[8];
    int32_t ch[5];
    double lam = 0.0;
    int64_t step = 0, n64 = 0;
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kNetMagic, 8) == 0 &&
              std::fread(ch, sizeof ch, 1, f) == 1 && std::fread(&lam, sizeof(double), 1, f) == 1 &&
              std::fread(&step, 8, 1, f) == 1 && std::fread(&n64, 8, 1, f) == 1;
    const long long nw = net->net.nweights();
    bool same = ok && n64 == nw;
    for (int l = 0; l < 5 && same; ++l) same = ch[l] == net->net.ch[l];
    std::vector<float> host;
    if (same) {
      host.resize(3 * nw);
      ok = std::fread(host.data(), sizeof(float), host.size(), f) == host.size();
    }
    std::fclose(f);
    need(ok, MGDWF_ERR_INVALID_ARG, "not a complete network file");
    need(same, MGDWF_ERR_STATE, "the file holds a network of other channel counts");
    net->net.set_weights(host.data(), nullptr);  // weights and their BF16 copy (resets Adam)
    MG_HIP(hipMemcpy(net->net.m.p, host.data() + nw, nw * sizeof(float), hipMemcpyHostToDevice));
    MG_HIP(hipMemcpy(net->net.v.p, host.data() + 2 * nw, nw * sizeof(float), hipMemcpyHostToDevice));
    net->net.step = step;
    net->net.lam = lam;
  });
}

}  // extern "C"
