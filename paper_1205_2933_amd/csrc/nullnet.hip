// Gauge-covariant proposal network for near-null vectors: forward, loss,
// backward and Adam, FP32 arithmetic with BF16 weights.
//
// The adaptive setup of the paper (Sec. 2) finds near-null vectors with a
// Krylov solver on A x = 0; this network proposes their 4D part from the gauge
// field, and the fifth dimension is the free-field wall profile (every low
// mode has the same fifth-dimension structure, Sec. 2 last paragraph).
//
//   layer:  out_o(x) = sum_{d, i} W[d][o][i] (T_d in_i)(x),  W real,
//           T_0 = 1, T_{1+2mu} f(x) = U_mu(x) f(x+mu), T_{2+2mu} f(x) = U_mu(x-mu)^+ f(x-mu)
//   gate:   g(f) = f a / (1 + a), a = |f(x)|^2 over colour (after layers 1..3)
//   output: channel 4k + alpha = spin alpha of proposal k
//   lift:   v_k(x, s) = P_+ f_k(x) w^(Ls-1-s) + P_- f_k(x) w^s, w = 1 - M5
//   loss:   mean_k |(1 - Pi) v_k|^2 / |v_k|^2 + lam mean_{j<k} |<f_j,f_k>|^2 / (|f_j|^2 |f_k|^2),
//           Pi = P R on the handle's installed basis.
//
// 4D channel fields are stored [channel][colour][x4] (float2), so a
// wavefront's lanes read consecutive sites.
#include <cmath>
#include <random>
#include <vector>

#include "blas.h"
#include "ctx.h"
#include "nullnet.h"

namespace mgdwf {

namespace {

struct Net4D {
  int L[4];
  int V4;
};

__device__ __forceinline__ void nbr(const Net4D& g, int x4, int mu, int& fwd, int& bwd) {
  int co[4];
  int r = x4;
  co[0] = r % g.L[0]; r /= g.L[0];
  co[1] = r % g.L[1]; r /= g.L[1];
  co[2] = r % g.L[2]; co[3] = r / g.L[2];
  const int st[4] = {1, g.L[0], g.L[0] * g.L[1], g.L[0] * g.L[1] * g.L[2]};
  fwd = co[mu] == g.L[mu] - 1 ? x4 - (g.L[mu] - 1) * st[mu] : x4 + st[mu];
  bwd = co[mu] == 0 ? x4 + (g.L[mu] - 1) * st[mu] : x4 - st[mu];
}

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __builtin_bit_cast(float, (uint32_t)b << 16); }
__device__ __forceinline__ uint16_t f32_to_bf16(float v) {
  uint32_t b = __builtin_bit_cast(uint32_t, v);
  if ((b & 0x7f800000u) == 0x7f800000u && (b & 0x007fffffu)) return (uint16_t)((b >> 16) | 0x40);
  b += 0x7fffu + ((b >> 16) & 1u);
  return (uint16_t)(b >> 16);
}

// y = U x (DAG false) or U^+ x, link (mu, a, b) at (mu*9 + a*3 + b) * V4 + x4
template <bool DAG>
__device__ __forceinline__ void link_mul(const float2* __restrict__ U, int mu, int V4, int x4, const float2 in[3],
                                         float2 out[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float2 s = make_float2(0.f, 0.f);
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      if (DAG) cfmac(s, U[(mu * 9 + b * 3 + a) * (long long)V4 + x4], in[b]);
      else cfma(s, U[(mu * 9 + a * 3 + b) * (long long)V4 + x4], in[b]);
    }
    out[a] = s;
  }
}

__device__ __forceinline__ void ld3(const float2* __restrict__ f, int ch, int V4, int x4, float2 v[3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) v[c] = f[((long long)ch * 3 + c) * V4 + x4];
}
__device__ __forceinline__ void st3(float2* __restrict__ f, int ch, int V4, int x4, const float2 v[3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) f[((long long)ch * 3 + c) * V4 + x4] = v[c];
}

// canonical complex128 [C][x4][3] -> internal float2 [C][3][x4]
__global__ void k_eta_pack(const double2* __restrict__ in, float2* __restrict__ out, int C, int V4) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)C * V4) return;
  const int ch = (int)(i / V4), x4 = (int)(i % V4);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double2 v = in[((long long)ch * V4 + x4) * 3 + c];
    out[((long long)ch * 3 + c) * V4 + x4] = make_float2((float)v.x, (float)v.y);
  }
}

// X[d * Cin + i] = T_d in_i, one thread per (x4, i)
__global__ void k_transport9(const float2* __restrict__ in, float2* __restrict__ X, const float2* __restrict__ U,
                             Net4D g, int Cin) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)Cin * g.V4) return;
  const int i = (int)(t / g.V4), x4 = (int)(t % g.V4);
  float2 v[3], w[3];
  ld3(in, i, g.V4, x4, v);
  st3(X, i, g.V4, x4, v);
  for (int mu = 0; mu < 4; ++mu) {
    int xf, xb;
    nbr(g, x4, mu, xf, xb);
    ld3(in, i, g.V4, xf, v);
    link_mul<false>(U, mu, g.V4, x4, v, w);            // U_mu(x) f(x+mu)
    st3(X, (1 + 2 * mu) * Cin + i, g.V4, x4, w);
    ld3(in, i, g.V4, xb, v);
    link_mul<true>(U, mu, g.V4, xb, v, w);             // U_mu(x-mu)^+ f(x-mu)
    st3(X, (2 + 2 * mu) * Cin + i, g.V4, x4, w);
  }
}

// gin_i = sum_d T_d^+ GX[d * Cin + i], T_d^+ = T_opposite(d); one thread per (x4, i)
__global__ void k_transport9_adj(const float2* __restrict__ GX, float2* __restrict__ gin, const float2* __restrict__ U,
                                 Net4D g, int Cin) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)Cin * g.V4) return;
  const int i = (int)(t / g.V4), x4 = (int)(t % g.V4);
  float2 acc[3], v[3], w[3];
  ld3(GX, i, g.V4, x4, acc);
  for (int mu = 0; mu < 4; ++mu) {
    int xf, xb;
    nbr(g, x4, mu, xf, xb);
    // the +mu hop's adjoint: U_mu(x-mu)^+ g(x-mu)
    ld3(GX, (1 + 2 * mu) * Cin + i, g.V4, xb, v);
    link_mul<true>(U, mu, g.V4, xb, v, w);
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[c] = cadd(acc[c], w[c]);
    // the -mu hop's adjoint: U_mu(x) g(x+mu)
    ld3(GX, (2 + 2 * mu) * Cin + i, g.V4, xf, v);
    link_mul<false>(U, mu, g.V4, x4, v, w);
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[c] = cadd(acc[c], w[c]);
  }
  st3(gin, i, g.V4, x4, acc);
}

// out_o = sum_j W[o][j] X_j over j < 9 Cin (W index (d * Cout + o) * Cin + i, j = d * Cin + i);
// one thread per (x4, o).  TRANS: GX_j = sum_o W[o][j] G_o, one thread per (x4, j).
template <bool TRANS>
__global__ void k_mix(const float2* __restrict__ in, float2* __restrict__ out, const uint16_t* __restrict__ W,
                      int V4, int Cin, int Cout) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int nout = TRANS ? 9 * Cin : Cout;
  if (t >= (long long)nout * V4) return;
  const int q = (int)(t / V4), x4 = (int)(t % V4);
  float2 acc[3] = {make_float2(0.f, 0.f), make_float2(0.f, 0.f), make_float2(0.f, 0.f)};
  if (!TRANS) {
    for (int j = 0; j < 9 * Cin; ++j) {
      const int d = j / Cin, i = j - d * Cin;
      const float w = bf16_to_f32(W[((long long)d * Cout + q) * Cin + i]);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float2 x = in[((long long)j * 3 + c) * V4 + x4];
        acc[c].x += w * x.x;
        acc[c].y += w * x.y;
      }
    }
  } else {
    const int d = q / Cin, i = q - d * Cin;
    for (int o = 0; o < Cout; ++o) {
      const float w = bf16_to_f32(W[((long long)d * Cout + o) * Cin + i]);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float2 x = in[((long long)o * 3 + c) * V4 + x4];
        acc[c].x += w * x.x;
        acc[c].y += w * x.y;
      }
    }
  }
  st3(out, q, V4, x4, acc);
}

// gate forward (post = pre a / (1 + a)) and backward (gpre from gpost), per (x4, channel)
template <bool BWD>
__global__ void k_gate(const float2* __restrict__ pre, const float2* __restrict__ gpost, float2* __restrict__ out,
                       int C, int V4) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)C * V4) return;
  const int ch = (int)(t / V4), x4 = (int)(t % V4);
  float2 f[3];
  ld3(pre, ch, V4, x4, f);
  const float a = f[0].x * f[0].x + f[0].y * f[0].y + f[1].x * f[1].x + f[1].y * f[1].y + f[2].x * f[2].x +
                  f[2].y * f[2].y;
  const float s = a / (1.f + a);
  float2 o[3];
  if (!BWD) {
#pragma unroll
    for (int c = 0; c < 3; ++c) o[c] = cscale(f[c], s);
  } else {
    float2 G[3];
    ld3(gpost, ch, V4, x4, G);
    float re = 0.f;
#pragma unroll
    for (int c = 0; c < 3; ++c) re += G[c].x * f[c].x + G[c].y * f[c].y;
    const float k2 = 2.f * re / ((1.f + a) * (1.f + a));
#pragma unroll
    for (int c = 0; c < 3; ++c) o[c] = make_float2(G[c].x * s + k2 * f[c].x, G[c].y * s + k2 * f[c].y);
  }
  st3(out, ch, V4, x4, o);
}

// dW[(d * Cout + o) * Cin + i] = sum_{x, c} Re(conj(G_o) X_{d Cin + i}); one workgroup per weight
__global__ __launch_bounds__(256) void k_gradW(const float2* __restrict__ G, const float2* __restrict__ X,
                                               float* __restrict__ dW, int V4, int Cin, int Cout) {
  const int widx = blockIdx.x;
  const int d = widx / (Cout * Cin), rem = widx % (Cout * Cin);
  const int o = rem / Cin, i = rem % Cin;
  const int j = d * Cin + i;
  double acc = 0.0;
  for (long long e = threadIdx.x; e < 3LL * V4; e += 256) {
    const float2 gv = G[(long long)o * 3 * V4 + e];
    const float2 xv = X[(long long)j * 3 * V4 + e];
    acc += (double)gv.x * xv.x + (double)gv.y * xv.y;
  }
  acc = block_sum<256>(acc);
  if (threadIdx.x == 0) dW[widx] = (float)acc;
}

// 4D spinor channels (4 nh) -> nh 5D fields in the fine layout (c * V4 + x4) * Ls + s
__global__ void k_lift(const float2* __restrict__ f, float2* __restrict__ v, int V4, int Ls, float w, int nh) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long V5 = (long long)V4 * Ls;
  if (t >= (long long)nh * V5) return;
  const int k = (int)(t / V5);
  const long long i5 = t % V5;
  const int x4 = (int)(i5 / Ls), s = (int)(i5 % Ls);
  const float wp = powf(w, (float)(Ls - 1 - s)), wm = powf(w, (float)s);
  for (int al = 0; al < 4; ++al)
    for (int c = 0; c < 3; ++c) {
      const float2 x = f[((long long)(4 * k + al) * 3 + c) * V4 + x4];
      v[(long long)k * 12 * V5 + (long long)(al * 3 + c) * V5 + i5] = cscale(x, al < 2 ? wp : wm);
    }
}

__global__ void k_lift_adj(const float2* __restrict__ g, float2* __restrict__ f, int V4, int Ls, float w, int nh) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)nh * 12 * V4) return;
  const int k = (int)(t / (12LL * V4));
  const int rem = (int)(t % (12LL * V4));
  const int cc = rem / V4, x4 = rem % V4;  // cc = alpha * 3 + colour
  const int al = cc / 3, c = cc % 3;
  const long long V5 = (long long)V4 * Ls;
  float2 acc = make_float2(0.f, 0.f);
  for (int s = 0; s < Ls; ++s) {
    const float ws = al < 2 ? powf(w, (float)(Ls - 1 - s)) : powf(w, (float)s);
    acc = cadd(acc, cscale(g[(long long)k * 12 * V5 + (long long)cc * V5 + (long long)x4 * Ls + s], ws));
  }
  f[((long long)(4 * k + al) * 3 + c) * V4 + x4] = acc;
}

// gv = -(2 / (N nh)) (pv - (Q / N) v), N = |v|^2 (slot 0), Q = |pv|^2 (slot 1) per RHS
__global__ void k_loss_grad_v(const float2* __restrict__ v, const float2* __restrict__ pv, float2* __restrict__ gv,
                              const double* __restrict__ sl, long long n, int nh, int nslot) {
  const int k = blockIdx.y;
  const double N = sl[k * nslot + 0], Q = sl[k * nslot + 1];
  const float a = (float)(-2.0 / (N * nh)), b = (float)(Q / N);
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const float2 x = v[k * n + i], p = pv[k * n + i];
    gv[k * n + i] = make_float2(a * (p.x - b * x.x), a * (p.y - b * x.y));
  }
}

// Gram matrix of the nh proposals f_k (channels 4k..4k+3): one workgroup per (j, k >= j)
__global__ __launch_bounds__(256) void k_gram(const float2* __restrict__ f, double* __restrict__ out, int V4, int nh) {
  const int j = blockIdx.x, k = blockIdx.y;
  if (k < j) return;
  const long long n = 12LL * V4;
  double re = 0.0, im = 0.0;
  for (long long e = threadIdx.x; e < n; e += 256) {
    const float2 a = f[(long long)j * n + e], b = f[(long long)k * n + e];
    re += (double)a.x * b.x + (double)a.y * b.y;
    im += (double)a.x * b.y - (double)a.y * b.x;
  }
  re = block_sum<256>(re);
  im = block_sum<256>(im);
  if (threadIdx.x == 0) { out[2 * (j * nh + k)] = re; out[2 * (j * nh + k) + 1] = im; }
}

// gf_j += sum_k A[j][k] f_k (complex coefficients, FP64 on input)
__global__ void k_gram_grad(const float2* __restrict__ f, float2* __restrict__ gf, const double* __restrict__ A,
                            int V4, int nh) {
  const long long n = 12LL * V4;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)nh * n) return;
  const int j = (int)(t / n);
  const long long e = t % n;
  float2 acc = gf[t];
  for (int k = 0; k < nh; ++k) {
    const float2 c = make_float2((float)A[2 * (j * nh + k)], (float)A[2 * (j * nh + k) + 1]);
    cfma(acc, c, f[(long long)k * n + e]);
  }
  gf[t] = acc;
}

__global__ void k_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v, const float* __restrict__ g,
                       uint16_t* __restrict__ wb, long long n, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  w[i] = wi;
  wb[i] = f32_to_bf16(wi);
}

__global__ void k_to_bf16(const float* __restrict__ w, uint16_t* __restrict__ wb, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) wb[i] = f32_to_bf16(w[i]);
}

int nb(long long n) { return ceil_div(n, 256); }

}  // namespace

long long NullNet::nweights() const {
  long long n = 0;
  for (int l = 0; l < 4; ++l) n += 9LL * ch[l] * ch[l + 1];
  return n;
}

long long NullNet::woff(int l) const {
  long long n = 0;
  for (int q = 0; q < l; ++q) n += 9LL * ch[q] * ch[q + 1];
  return n;
}

// Weights of layer l drawn from N(0, 1 / (9 C_in)) (seeded), so that a layer
// keeps the colour norm of unit-variance inputs and the gate starts near its
// linear regime.
void NullNet::init(unsigned long long seed) {
  const long long n = nweights();
  w.alloc(n * sizeof(float));
  wb.alloc(n * sizeof(uint16_t));
  m.alloc(n * sizeof(float));
  v.alloc(n * sizeof(float));
  g.alloc(n * sizeof(float));
  std::vector<float> host((size_t)n);
  std::mt19937_64 rng(seed);
  std::normal_distribution<float> nd(0.f, 1.f);
  for (int l = 0; l < 4; ++l) {
    const float sd = 1.f / std::sqrt(9.f * ch[l]);
    for (long long i = woff(l); i < woff(l) + 9LL * ch[l] * ch[l + 1]; ++i) host[(size_t)i] = sd * nd(rng);
  }
  set_weights(host.data(), nullptr);
}

void NullNet::set_weights(const float* host, hipStream_t st) {
  const long long n = nweights();
  MG_HIP(hipMemcpyAsync(w.p, host, n * sizeof(float), hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_to_bf16, dim3(nb(n)), dim3(256), 0, st, w.as<float>(), wb.as<uint16_t>(), n);
  MG_LAUNCH_CHECK();
  MG_HIP(hipMemsetAsync(m.p, 0, n * sizeof(float), st));
  MG_HIP(hipMemsetAsync(v.p, 0, n * sizeof(float), st));
  MG_HIP(hipStreamSynchronize(st));
  step = 0;
}

// Forward pass on the handle's lattice; keeps every layer's input transports
// (X_l), pre-activations and outputs in the handle's workspace for backward.
static void net_forward(NullNet& net, mgdwf_ctx* c, const double2* eta_canon) {
  const int V4 = c->g.V4;
  Net4D g4;
  for (int m = 0; m < 4; ++m) g4.L[m] = c->g.L[m];
  g4.V4 = V4;
  const long long f1 = 3LL * V4;  // one channel
  float2* h = c->buf<float2>("nn_h0", net.ch[0] * f1);
  hipLaunchKernelGGL(k_eta_pack, dim3(nb((long long)net.ch[0] * V4)), dim3(256), 0, c->st, eta_canon, h, net.ch[0], V4);
  MG_LAUNCH_CHECK();
  const float2* U = c->U32.as<float2>();
  for (int l = 0; l < 4; ++l) {
    const int Cin = net.ch[l], Cout = net.ch[l + 1];
    const std::string tag = std::to_string(l);
    float2* X = c->buf<float2>("nn_X" + tag, 9LL * Cin * f1);
    float2* pre = c->buf<float2>("nn_pre" + tag, Cout * f1);
    hipLaunchKernelGGL(k_transport9, dim3(nb((long long)Cin * V4)), dim3(256), 0, c->st, h, X, U, g4, Cin);
    MG_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_mix<false>, dim3(nb((long long)Cout * V4)), dim3(256), 0, c->st, X, pre,
                       net.wb.as<uint16_t>() + net.woff(l), V4, Cin, Cout);
    MG_LAUNCH_CHECK();
    if (l < 3) {
      float2* post = c->buf<float2>("nn_h" + std::to_string(l + 1), Cout * f1);
      hipLaunchKernelGGL(k_gate<false>, dim3(nb((long long)Cout * V4)), dim3(256), 0, c->st, pre, nullptr, post, Cout, V4);
      MG_LAUNCH_CHECK();
      h = post;
    }
  }
}

void net_propose(NullNet& net, mgdwf_ctx* c, const double2* eta, double2* V_canon) {
  net_forward(net, c, eta);
  const int V4 = c->g.V4, Ls = c->g.Ls, nh = net.ch[4] / 4;
  const long long nf = c->fine_len();
  float2* v32 = c->buf<float2>("nn_v", nf * nh);
  hipLaunchKernelGGL(k_lift, dim3(nb((long long)nh * V4 * Ls)), dim3(256), 0, c->st, c->buf<float2>("nn_pre3", 0),
                     v32, V4, Ls, (float)(1.0 - c->M5), nh);
  MG_LAUNCH_CHECK();
  double2* v64 = c->buf<double2>("nn_v64", nf * nh);
  convert<float2, double2>(v32, v64, nf * nh, c->st);
  unpack_fermion_f64(v64, V_canon, c->g, nh, c->st);
  MG_HIP(hipStreamSynchronize(c->st));
}

// Loss and weight gradient (into net.g) against the handle's installed basis.
double net_grad(NullNet& net, mgdwf_ctx* c, const double2* eta) {
  if (!c->have_basis) fail(MGDWF_ERR_STATE, "install a target basis (set_nullvecs) first");
  net_forward(net, c, eta);
  const int V4 = c->g.V4, Ls = c->g.Ls, nh = net.ch[4] / 4;
  const float w = (float)(1.0 - c->M5);
  const long long nf = c->fine_len(), f1 = 3LL * V4;
  float2* out = c->buf<float2>("nn_pre3", 0);
  float2* v = c->buf<float2>("nn_v", nf * nh);
  float2* pv = c->buf<float2>("nn_pv", nf * nh);
  float2* gv = c->buf<float2>("nn_gv", nf * nh);
  float2* cv = c->buf<float2>("nn_cv", (long long)c->coarse_len() * nh);
  hipLaunchKernelGGL(k_lift, dim3(nb((long long)nh * V4 * Ls)), dim3(256), 0, c->st, out, v, V4, Ls, w, nh);
  MG_LAUNCH_CHECK();
  restrict_op<float2, float2>(c->V32.as<float2>(), v, cv, c->buf<double>("rpart", restrict_partial_doubles(c->cg, nh)),
                              c->g, c->cg, nh, c->st);
  prolong_op<float2, float2>(c->V32.as<float2>(), cv, pv, false, c->g, c->cg, nh, c->st);
  // per-proposal |v|^2 and |Pi v|^2 into two slots of a small table
  double* sl = c->buf<double>("nn_slots", (size_t)nh * NSLOT);
  double* part = c->buf<double>("vpart", (size_t)VEC_BLOCKS * nh * (2 * 16 + 3));
  multidot_rhs<float2>(nullptr, 0, v, nullptr, nf, nh, part, sl, 0, c->st);
  multidot_rhs<float2>(nullptr, 0, pv, nullptr, nf, nh, part, sl, 1, c->st);  // after slot 0: |Pi v|^2 in slot 1
  hipLaunchKernelGGL(k_loss_grad_v, dim3(std::min(nb(nf), VEC_BLOCKS), nh), dim3(256), 0, c->st, v, pv, gv, sl, nf, nh,
                     NSLOT);
  MG_LAUNCH_CHECK();
  // gradient with respect to the output channels: lift adjoint + Gram term
  float2* gout = c->buf<float2>("nn_g3", (long long)net.ch[4] * f1);
  hipLaunchKernelGGL(k_lift_adj, dim3(nb((long long)nh * 12 * V4)), dim3(256), 0, c->st, gv, gout, V4, Ls, w, nh);
  MG_LAUNCH_CHECK();
  double* gram = c->buf<double>("nn_gram", 2LL * nh * nh);
  hipLaunchKernelGGL(k_gram, dim3(nh, nh), dim3(256), 0, c->st, out, gram, V4, nh);
  MG_LAUNCH_CHECK();
  std::vector<double> hs((size_t)nh * NSLOT), G(2LL * nh * nh);
  MG_HIP(hipMemcpyAsync(hs.data(), sl, hs.size() * sizeof(double), hipMemcpyDeviceToHost, c->st));
  MG_HIP(hipMemcpyAsync(G.data(), gram, G.size() * sizeof(double), hipMemcpyDeviceToHost, c->st));
  MG_HIP(hipStreamSynchronize(c->st));
  double loss = 0.0;
  for (int k = 0; k < nh; ++k) loss += (1.0 - hs[k * NSLOT + 1] / hs[k * NSLOT + 0]) / nh;
  std::vector<double> A(2LL * nh * nh, 0.0);
  const double npair = nh * (nh - 1) / 2.0;
  auto gr = [&](int j, int k) { return G[2 * (j * nh + k)]; };
  auto gi = [&](int j, int k) { return G[2 * (j * nh + k) + 1]; };
  for (int j = 0; j < nh; ++j)
    for (int k = j + 1; k < nh; ++k) {
      const double cr = gr(j, k), ci = gi(j, k), Nj = gr(j, j), Nk = gr(k, k);
      const double a2 = cr * cr + ci * ci;
      loss += net.lam * a2 / (Nj * Nk) / npair;
      const double sc = net.lam * 2.0 / (Nj * Nk) / npair;
      // gf_j += sc (conj(c) f_k - a2/Nj f_j);  gf_k += sc (c f_j - a2/Nk f_k)
      A[2 * (j * nh + k)] += sc * cr;
      A[2 * (j * nh + k) + 1] += -sc * ci;
      A[2 * (j * nh + j)] += -sc * a2 / Nj;
      A[2 * (k * nh + j)] += sc * cr;
      A[2 * (k * nh + j) + 1] += sc * ci;
      A[2 * (k * nh + k)] += -sc * a2 / Nk;
    }
  double* Ad = c->buf<double>("nn_A", A.size());
  MG_HIP(hipMemcpyAsync(Ad, A.data(), A.size() * sizeof(double), hipMemcpyHostToDevice, c->st));
  hipLaunchKernelGGL(k_gram_grad, dim3(nb((long long)nh * 12 * V4)), dim3(256), 0, c->st, out, gout, Ad, V4, nh);
  MG_LAUNCH_CHECK();
  // backward through the layers
  Net4D g4;
  for (int m = 0; m < 4; ++m) g4.L[m] = c->g.L[m];
  g4.V4 = V4;
  const float2* U = c->U32.as<float2>();
  float2* gcur = gout;
  for (int l = 3; l >= 0; --l) {
    const int Cin = net.ch[l], Cout = net.ch[l + 1];
    const std::string tag = std::to_string(l);
    float2* pre = c->buf<float2>("nn_pre" + tag, 0);
    float2* X = c->buf<float2>("nn_X" + tag, 0);
    if (l < 3) {
      float2* gp = c->buf<float2>("nn_gpre", (long long)Cout * f1);
      hipLaunchKernelGGL(k_gate<true>, dim3(nb((long long)Cout * V4)), dim3(256), 0, c->st, pre, gcur, gp, Cout, V4);
      MG_LAUNCH_CHECK();
      gcur = gp;
    }
    hipLaunchKernelGGL(k_gradW, dim3(9 * Cin * Cout), dim3(256), 0, c->st, gcur, X, net.g.as<float>() + net.woff(l),
                       V4, Cin, Cout);
    MG_LAUNCH_CHECK();
    if (l > 0) {
      float2* GX = c->buf<float2>("nn_GX", 9LL * Cin * f1);
      hipLaunchKernelGGL(k_mix<true>, dim3(nb(9LL * Cin * V4)), dim3(256), 0, c->st, gcur, GX,
                         net.wb.as<uint16_t>() + net.woff(l), V4, Cin, Cout);
      MG_LAUNCH_CHECK();
      float2* gin = c->buf<float2>(std::string("nn_gin") + (l % 2 ? "a" : "b"), (long long)Cin * f1);
      hipLaunchKernelGGL(k_transport9_adj, dim3(nb((long long)Cin * V4)), dim3(256), 0, c->st, GX, gin, U, g4, Cin);
      MG_LAUNCH_CHECK();
      gcur = gin;
    }
  }
  MG_HIP(hipStreamSynchronize(c->st));
  return loss;
}

double net_train_step(NullNet& net, mgdwf_ctx* c, const double2* eta, double lr) {
  const double loss = net_grad(net, c, eta);
  const long long n = net.nweights();
  net.step += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - std::pow(b1, (float)net.step), c2 = 1.f - std::pow(b2, (float)net.step);
  hipLaunchKernelGGL(k_adam, dim3(nb(n)), dim3(256), 0, c->st, net.w.as<float>(), net.m.as<float>(), net.v.as<float>(),
                     net.g.as<float>(), net.wb.as<uint16_t>(), n, (float)lr, b1, b2, 1e-8f, c1, c2);
  MG_LAUNCH_CHECK();
  MG_HIP(hipStreamSynchronize(c->st));
  return loss;
}

}  // namespace mgdwf
