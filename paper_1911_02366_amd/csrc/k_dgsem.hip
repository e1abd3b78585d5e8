// Nonlinear residual of the backward-Euler GL-DGSEM step on the device:
//     R(Q) = M (Q - Q_s) / dt + H(Q)
// for the compressible Navier-Stokes equations on a periodic Cartesian hex
// mesh (paper, eq. ImplicitDisc; H from eq. DGSEMsystem: weak form on
// Gauss-Lobatto nodes, local Lax-Friedrichs advective flux, Bassi-Rebay 1
// viscous flux with the lifted gradient of eq. DGSEMsystem:2).
//
// Two launches, one workgroup per element, one thread per node:
//   1. lifted gradient g_d (strong form):
//        g_d = s [ sum_a D[l][a] q_a + (1/w_N) [l = N] (q^+_R - q_N)/2 - (1/w_0) [l = 0] (q^-_L - q_0)/2 ]
//   2. residual: fluxes F_d = f^a_d(q) - f^nu_d(q, g) staged in LDS, then
//        H = J s w_i w_j w_k sum_d (1/w_l) [ sum_a Vw[l][a] F_d(a) + [l = N] Fhat_R - [l = 0] Fhat_L ]
//      with Vw[l][a] = -w_a D[a][l] and Fhat = LLF(q_L, q_R) - (f^nu(q_L, g_L) + f^nu(q_R, g_R)) / 2.
// A face flux is evaluated by both elements with identical arguments, so the
// scheme stays conservative to the last bit.
//
// The Newton matrix of eq. NewtonLinSys1 applied to a vector,
//     A v = M v / dt + dH/dQ(Q) v,
// runs the same two launches on dual numbers (forward-mode differentiation):
// the lifting is linear, so the direction's gradient is the lifting of v, and
// the residual sums carry value and derivative; only the derivative is kept.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <type_traits>
#include <vector>

#include "internal.hpp"

namespace scdg {

namespace {

constexpr int kMaxP = kMaxOrder + 1;

struct DgParams {
  int k_elem, p;
  int sipg;                  // 1: interior-penalty face viscous flux (else Bassi-Rebay 1)
  double s, jac, gamma, mach2, inv_re, prandtl, suth;
  double sigma;              // interior-penalty factor eta (N + 1)^2 / h
  double w[kMaxP];
  double d[kMaxP][kMaxP];    // D[l][a] = l_a'(x_l)
  double vw[kMaxP][kMaxP];   // -w_a D[a][l]
};

// Forward-mode dual number: a value and its derivative along one direction
// of the state.  Evaluating the residual on duals gives dH/dQ v exactly to
// rounding, with no step size.  |x| passes on sign(x) x' (zero at x = 0) and
// the larger of the two Lax-Friedrichs speeds passes on the derivative of the
// one selected (the left one at a tie), the same branches as the residual.
struct Dual {
  double v, d;
  Dual() = default;
  __device__ Dual(double a) : v(a), d(0.0) {}
  __device__ Dual(double a, double b) : v(a), d(b) {}
};
__device__ __forceinline__ Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
__device__ __forceinline__ Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
__device__ __forceinline__ Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
__device__ __forceinline__ Dual operator/(Dual a, Dual b) {
  const double r = a.v / b.v;
  return Dual(r, (a.d - r * b.d) / b.v);
}
__device__ __forceinline__ Dual &operator+=(Dual &a, Dual b) { return a = a + b; }
__device__ __forceinline__ Dual &operator-=(Dual &a, Dual b) { return a = a - b; }
__device__ __forceinline__ bool operator>=(Dual a, Dual b) { return a.v >= b.v; }
__device__ __forceinline__ double vsqrt(double x) { return ::sqrt(x); }
__device__ __forceinline__ Dual vsqrt(Dual x) {
  const double r = ::sqrt(x.v);
  return Dual(r, 0.5 * x.d / r);
}
__device__ __forceinline__ double vabs(double x) { return ::fabs(x); }
__device__ __forceinline__ Dual vabs(Dual x) {
  const double sg = x.v > 0.0 ? 1.0 : (x.v < 0.0 ? -1.0 : 0.0);
  return Dual(sg * x.v, sg * x.d);
}
// what the volume and surface sums carry: the value, or the derivative alone
__device__ __forceinline__ double part(double x) { return x; }
__device__ __forceinline__ double part(Dual x) { return x.d; }
// element i of a state-like array: the value, or value and direction
template <class T>
__device__ __forceinline__ T at(const double *x, const double *dx, int64_t i);
template <>
__device__ __forceinline__ double at<double>(const double *x, const double *, int64_t i) {
  return x[i];
}
template <>
__device__ __forceinline__ Dual at<Dual>(const double *x, const double *dx, int64_t i) {
  return Dual(x[i], dx[i]);
}

template <class T>
struct Prim {
  T rho, u[3], p, e;  // e: specific internal energy
};

template <class T>
__device__ __forceinline__ Prim<T> prim(const T q[5], double gamma) {
  Prim<T> r;
  r.rho = q[0];
  const T ir = 1.0 / q[0];
  r.u[0] = q[1] * ir;
  r.u[1] = q[2] * ir;
  r.u[2] = q[3] * ir;
  const T ke = 0.5 * (r.u[0] * r.u[0] + r.u[1] * r.u[1] + r.u[2] * r.u[2]);
  r.e = q[4] * ir - ke;
  r.p = (gamma - 1.0) * q[0] * r.e;
  return r;
}

template <class T>
__device__ void flux_adv(const T q[5], int d, double gamma, T f[5]) {
  const Prim<T> a = prim(q, gamma);
  const T vd = a.u[d];
  f[0] = q[0] * vd;
  f[1] = q[1] * vd;
  f[2] = q[2] * vd;
  f[3] = q[3] * vd;
  f[1 + d] += a.p;
  f[4] = vd * (q[4] + a.p);
}

// viscous flux f^nu_d(q, g); g[k*5 + v] = d q_v / d x_k
template <class T>
__device__ void flux_visc(const T q[5], const T g[15], int d, const DgParams &P, T f[5]) {
  const Prim<T> a = prim(q, P.gamma);
  const T ir = 1.0 / q[0];
  T dv[3][3];   // dv[i][k] = d u_i / d x_k
  T de[3];
  const T eE = q[4] * ir;
  for (int k = 0; k < 3; ++k) {
    for (int i = 0; i < 3; ++i) dv[i][k] = (g[k * 5 + 1 + i] - a.u[i] * g[k * 5]) * ir;
    de[k] = (g[k * 5 + 4] - eE * g[k * 5]) * ir -
            (a.u[0] * dv[0][k] + a.u[1] * dv[1][k] + a.u[2] * dv[2][k]);
  }
  const T temp = P.gamma * P.mach2 * a.p / q[0];
  const T mu = (1.0 + P.suth) / (temp + P.suth) * temp * vsqrt(temp);
  const T div = dv[0][0] + dv[1][1] + dv[2][2];
  T tau[3];
  for (int i = 0; i < 3; ++i) {
    tau[i] = mu * (dv[i][d] + dv[d][i]);
    if (i == d) tau[i] -= (2.0 / 3.0) * mu * div;
  }
  const T heat = mu * P.gamma / P.prandtl * de[d];
  f[0] = 0.0;
  f[1] = tau[0] * P.inv_re;
  f[2] = tau[1] * P.inv_re;
  f[3] = tau[2] * P.inv_re;
  f[4] = (a.u[0] * tau[0] + a.u[1] * tau[1] + a.u[2] * tau[2] + heat) * P.inv_re;
}

// total numerical flux through a +e_d face: LLF advective minus BR1 viscous
template <class T>
__device__ void face_flux(const T ql[5], const T gl[15], const T qr[5], const T gr[15], int d,
                          const DgParams &P, T fh[5]) {
  T fl[5], fr[5], vl[5], vr[5];
  flux_adv(ql, d, P.gamma, fl);
  flux_adv(qr, d, P.gamma, fr);
  const Prim<T> a = prim(ql, P.gamma), b = prim(qr, P.gamma);
  const T lam_l = vabs(a.u[d]) + vsqrt(P.gamma * a.p / a.rho);
  const T lam_r = vabs(b.u[d]) + vsqrt(P.gamma * b.p / b.rho);
  const T lam = lam_l >= lam_r ? lam_l : lam_r;
  flux_visc(ql, gl, d, P, vl);
  flux_visc(qr, gr, d, P, vr);
  for (int v = 0; v < 5; ++v)
    fh[v] = 0.5 * (fl[v] + fr[v]) - 0.5 * lam * (qr[v] - ql[v]) - 0.5 * (vl[v] + vr[v]);
}

// total numerical flux through a +e_d face with the symmetric interior penalty
// viscous flux: LLF advective minus
//   {{f^nu_d(q, grad q)}} + sigma f^nu_d({{q}}, [[q]] e_d),
// grad q the broken (element-local) gradients bl, br of the two sides and
// [[q]] = qr - ql taken as a gradient along the face normal
template <class T>
__device__ void face_flux_sipg(const T ql[5], const T bl[15], const T qr[5], const T br[15], int d,
                               const DgParams &P, T fh[5]) {
  T fl[5], fr[5], vl[5], vr[5], vp[5], qm[5], jg[15];
  flux_adv(ql, d, P.gamma, fl);
  flux_adv(qr, d, P.gamma, fr);
  const Prim<T> a = prim(ql, P.gamma), b = prim(qr, P.gamma);
  const T lam_l = vabs(a.u[d]) + vsqrt(P.gamma * a.p / a.rho);
  const T lam_r = vabs(b.u[d]) + vsqrt(P.gamma * b.p / b.rho);
  const T lam = lam_l >= lam_r ? lam_l : lam_r;
  flux_visc(ql, bl, d, P, vl);
  flux_visc(qr, br, d, P, vr);
  for (int t = 0; t < 15; ++t) jg[t] = 0.0;
  for (int v = 0; v < 5; ++v) {
    qm[v] = 0.5 * (ql[v] + qr[v]);
    jg[d * 5 + v] = qr[v] - ql[v];
  }
  flux_visc(qm, jg, d, P, vp);
  for (int v = 0; v < 5; ++v)
    fh[v] = 0.5 * (fl[v] + fr[v]) - 0.5 * lam * (qr[v] - ql[v]) - 0.5 * (vl[v] + vr[v]) - P.sigma * vp[v];
}

// total numerical flux along the unnormalized face normal nv (curved faces):
// sum_d nv_d {{f^a_d}} - lambda |nv| [[q]] / 2 - sum_d nv_d {{f^nu_d}},
// lambda the larger of |v . nv| / |nv| + c on the two sides
template <class T>
__device__ void face_flux_normal(const T ql[5], const T gl[15], const T qr[5], const T gr[15],
                                 const double nv[3], const DgParams &P, T fh[5]) {
  const double sn = sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
  const double inv = 1.0 / sn;
  const Prim<T> a = prim(ql, P.gamma), b = prim(qr, P.gamma);
  const T un_l = (a.u[0] * nv[0] + a.u[1] * nv[1] + a.u[2] * nv[2]) * inv;
  const T un_r = (b.u[0] * nv[0] + b.u[1] * nv[1] + b.u[2] * nv[2]) * inv;
  const T lam_l = vabs(un_l) + vsqrt(P.gamma * a.p / a.rho);
  const T lam_r = vabs(un_r) + vsqrt(P.gamma * b.p / b.rho);
  const T lam = lam_l >= lam_r ? lam_l : lam_r;
  T acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int d = 0; d < 3; ++d) {
    T fl[5], fr[5], vl[5], vr[5];
    flux_adv(ql, d, P.gamma, fl);
    flux_adv(qr, d, P.gamma, fr);
    flux_visc(ql, gl, d, P, vl);
    flux_visc(qr, gr, d, P, vr);
    for (int v = 0; v < 5; ++v) acc[v] += nv[d] * (0.5 * (fl[v] + fr[v]) - 0.5 * (vl[v] + vr[v]));
  }
  for (int v = 0; v < 5; ++v) fh[v] = acc[v] - 0.5 * lam * sn * (qr[v] - ql[v]);
}

// cooperative copy of the parameter block into LDS (ends with a barrier)
__device__ __forceinline__ void load_params(const DgParams *__restrict__ src, DgParams *dst) {
  static_assert(sizeof(DgParams) % 4 == 0, "word copy");
  const uint32_t *s = reinterpret_cast<const uint32_t *>(src);
  uint32_t *d = reinterpret_cast<uint32_t *>(dst);
  for (int t = threadIdx.x; t < (int)(sizeof(DgParams) / 4); t += blockDim.x) d[t] = s[t];
  __syncthreads();
}

__device__ __forceinline__ int nbr_elem(int e, int k, int d, int step) {
  int c[3] = {e % k, (e / k) % k, e / (k * k)};
  c[d] = (c[d] + step + k) % k;
  return c[0] + k * c[1] + k * k * c[2];
}

__device__ __forceinline__ int node_with(int node, int p, int d, int l) {
  int c[3] = {node % p, (node / p) % p, node / (p * p)};
  c[d] = l;
  return c[0] + p * c[1] + p * p * c[2];
}

// BR1 lifted gradient g; with gb != NULL also the broken gradient of each
// element's own interpolant (the same line derivatives without the surface term)
__global__ __launch_bounds__(512) void lift_kernel(const DgParams *__restrict__ prm, const double *__restrict__ q,
                            double *__restrict__ g, double *__restrict__ gb) {
  __shared__ DgParams P;
  __shared__ double qs[kMaxP * kMaxP * kMaxP * 5];
  load_params(prm, &P);
  const int p = P.p, p3 = p * p * p, n = p - 1;
  const int e = blockIdx.x;
  const double *qe = q + (int64_t)e * p3 * 5;
  for (int t = threadIdx.x; t < p3 * 5; t += blockDim.x) qs[t] = qe[t];
  __syncthreads();
  const int node = threadIdx.x;
  if (node >= p3) return;
  const int c[3] = {node % p, (node / p) % p, node / (p * p)};
  double out[15];
  for (int d = 0; d < 3; ++d) {
    const int l = c[d];
    for (int v = 0; v < 5; ++v) {
      double acc = 0.0;
      for (int a = 0; a < p; ++a) acc += P.d[l][a] * qs[node_with(node, p, d, a) * 5 + v];
      out[d * 5 + v] = acc;
    }
    if (gb) {
      double *gbe = gb + ((int64_t)e * p3 + node) * 15 + d * 5;
      for (int v = 0; v < 5; ++v) gbe[v] = P.s * out[d * 5 + v];
    }
    if (l == n) {
      const double *qn = q + ((int64_t)nbr_elem(e, P.k_elem, d, 1) * p3 + node_with(node, p, d, 0)) * 5;
      for (int v = 0; v < 5; ++v) out[d * 5 + v] += (0.5 / P.w[n]) * (qn[v] - qs[node * 5 + v]);
    }
    if (l == 0) {
      const double *qn = q + ((int64_t)nbr_elem(e, P.k_elem, d, -1) * p3 + node_with(node, p, d, n)) * 5;
      for (int v = 0; v < 5; ++v) out[d * 5 + v] -= (0.5 / P.w[0]) * (qn[v] - qs[node * 5 + v]);
    }
  }
  double *ge = g + ((int64_t)e * p3 + node) * 15;
  for (int t = 0; t < 15; ++t) ge[t] = P.s * out[t];
}

// Lifted gradient on curved elements (metric met: 10 doubles per node, (J a^i)_n
// at 3 i + n and J at 9):
//   g_n = (1/J) sum_i [ sum_a D[l][a] ((J a^i)_n q)_a
//                      + (1/w_N) [l = N] (J a^i)_n (q^+ - q) / 2 - (1/w_0) [l = 0] (J a^i)_n (q^- - q) / 2 ]
__global__ __launch_bounds__(512) void lift_curved_kernel(const DgParams *__restrict__ prm,
                                                          const double *__restrict__ q,
                                                          const double *__restrict__ met,
                                                          double *__restrict__ g) {
  __shared__ DgParams P;
  __shared__ double qs[kMaxP * kMaxP * kMaxP * 5];
  extern __shared__ double ms[];   // [p3][10] metric of the element
  load_params(prm, &P);
  const int p = P.p, p3 = p * p * p, n = p - 1;
  const int e = blockIdx.x;
  const double *qe = q + (int64_t)e * p3 * 5;
  const double *me = met + (int64_t)e * p3 * 10;
  for (int t = threadIdx.x; t < p3 * 5; t += blockDim.x) qs[t] = qe[t];
  for (int t = threadIdx.x; t < p3 * 10; t += blockDim.x) ms[t] = me[t];
  __syncthreads();
  const int node = threadIdx.x;
  if (node >= p3) return;
  const int c[3] = {node % p, (node / p) % p, node / (p * p)};
  double out[15];
  for (int t = 0; t < 15; ++t) out[t] = 0.0;
  for (int i = 0; i < 3; ++i) {
    const int l = c[i];
    for (int a = 0; a < p; ++a) {
      const int na = node_with(node, p, i, a);
      const double dl = P.d[l][a];
      for (int m = 0; m < 3; ++m) {
        const double f = dl * ms[na * 10 + 3 * i + m];
        for (int v = 0; v < 5; ++v) out[m * 5 + v] += f * qs[na * 5 + v];
      }
    }
    if (l == n || l == 0) {
      const int step = l == n ? 1 : -1;
      const double *qn = q + ((int64_t)nbr_elem(e, P.k_elem, i, step) * p3 + node_with(node, p, i, l == n ? 0 : n)) * 5;
      const double sgn = l == n ? 0.5 / P.w[n] : -0.5 / P.w[0];
      for (int m = 0; m < 3; ++m) {
        const double f = sgn * ms[node * 10 + 3 * i + m];
        for (int v = 0; v < 5; ++v) out[m * 5 + v] += f * (qn[v] - qs[node * 5 + v]);
      }
    }
  }
  const double inv_j = 1.0 / ms[node * 10 + 9];
  double *ge = g + ((int64_t)e * p3 + node) * 15;
  for (int t = 0; t < 15; ++t) ge[t] = inv_j * out[t];
}

// Residual on curved elements: contravariant fluxes F^i = sum_n (J a^i)_n f_n in
// LDS, the weak volume term and the face fluxes along J a^i of this element's
// face node, mass J w_i w_j w_k:
//   H = w_i w_j w_k sum_i (1/w_l) [ sum_a Vw[l][a] F^i(a) + [l = N] Fhat_R - [l = 0] Fhat_L ]
//
// With T = Dual the same sums give the directional derivative: q and g carry
// the direction dq and the lifted gradient of dq (the lifting is linear), and
// r = M inv_dt dq + dH/dQ(q) dq (q_s unused).
template <class T>
__global__ __launch_bounds__(512) void residual_curved_kernel(const DgParams *__restrict__ prm,
                                                              const double *__restrict__ q,
                                                              const double *__restrict__ dq,
                                                              const double *__restrict__ g,
                                                              const double *__restrict__ dg,
                                                              const double *__restrict__ met,
                                                              const double *__restrict__ q_s, double inv_dt,
                                                              double *__restrict__ r) {
  __shared__ DgParams P;
  extern __shared__ double fs[];   // [3][p3][5] contravariant fluxes
  load_params(prm, &P);
  const int p = P.p, p3 = p * p * p, n = p - 1;
  const int e = blockIdx.x;
  const int node = threadIdx.x;
  const bool live = node < p3;
  T qn[5], gn[15];
  double mn[10];
  if (live) {
    const int64_t id = (int64_t)e * p3 + node;
    for (int v = 0; v < 5; ++v) qn[v] = at<T>(q, dq, id * 5 + v);
    for (int t = 0; t < 15; ++t) gn[t] = at<T>(g, dg, id * 15 + t);
    for (int t = 0; t < 10; ++t) mn[t] = met[id * 10 + t];
    double ft[3][5];
    for (int i = 0; i < 3; ++i)
      for (int v = 0; v < 5; ++v) ft[i][v] = 0.0;
    for (int d = 0; d < 3; ++d) {
      T fa[5], fv[5];
      flux_adv(qn, d, P.gamma, fa);
      flux_visc(qn, gn, d, P, fv);
      for (int i = 0; i < 3; ++i)
        for (int v = 0; v < 5; ++v) ft[i][v] += mn[3 * i + d] * part(fa[v] - fv[v]);
    }
    for (int i = 0; i < 3; ++i)
      for (int v = 0; v < 5; ++v) fs[(i * p3 + node) * 5 + v] = ft[i][v];
  }
  __syncthreads();
  if (!live) return;
  const int c[3] = {node % p, (node / p) % p, node / (p * p)};
  double h[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int i = 0; i < 3; ++i) {
    const int l = c[i];
    double rd[5];
    for (int v = 0; v < 5; ++v) {
      double acc = 0.0;
      for (int a = 0; a < p; ++a) acc += P.vw[l][a] * fs[(i * p3 + node_with(node, p, i, a)) * 5 + v];
      rd[v] = acc;
    }
    const double nv[3] = {mn[3 * i], mn[3 * i + 1], mn[3 * i + 2]};
    if (l == n) {
      const int64_t nb = (int64_t)nbr_elem(e, P.k_elem, i, 1) * p3 + node_with(node, p, i, 0);
      T qb[5], gb[15], fh[5];
      for (int v = 0; v < 5; ++v) qb[v] = at<T>(q, dq, nb * 5 + v);
      for (int t = 0; t < 15; ++t) gb[t] = at<T>(g, dg, nb * 15 + t);
      face_flux_normal(qn, gn, qb, gb, nv, P, fh);
      for (int v = 0; v < 5; ++v) rd[v] += part(fh[v]);
    }
    if (l == 0) {
      const int64_t nb = (int64_t)nbr_elem(e, P.k_elem, i, -1) * p3 + node_with(node, p, i, n);
      T qb[5], gb[15], fh[5];
      for (int v = 0; v < 5; ++v) qb[v] = at<T>(q, dq, nb * 5 + v);
      for (int t = 0; t < 15; ++t) gb[t] = at<T>(g, dg, nb * 15 + t);
      face_flux_normal(qb, gb, qn, gn, nv, P, fh);
      for (int v = 0; v < 5; ++v) rd[v] -= part(fh[v]);
    }
    for (int v = 0; v < 5; ++v) h[v] += rd[v] / P.w[l];
  }
  const double w3 = P.w[c[0]] * P.w[c[1]] * P.w[c[2]];
  const double m = mn[9] * w3;
  const int64_t id = (int64_t)e * p3 + node;
  double *re = r + id * 5;
  for (int v = 0; v < 5; ++v) {
    double val = w3 * h[v];
    if constexpr (std::is_same<T, Dual>::value) {
      val += m * inv_dt * dq[id * 5 + v];
    } else {
      if (q_s) val += m * inv_dt * (qn[v] - q_s[id * 5 + v]);
    }
    re[v] = val;
  }
}

// With T = Dual: r = M inv_dt dq + dH/dQ(q) dq, dg the lifted gradient of dq.
// SIPG: the face viscous flux is the interior-penalty flux on the broken
// gradients gbq (dgb for the direction); a template argument, so that the
// Bassi-Rebay 1 kernels carry none of its code.
template <class T, bool SIPG>
__global__ __launch_bounds__(512) void residual_kernel(const DgParams *__restrict__ prm, const double *__restrict__ q,
                                const double *__restrict__ dq, const double *__restrict__ g,
                                const double *__restrict__ dg, const double *__restrict__ gbq,
                                const double *__restrict__ dgb, const double *__restrict__ q_s,
                                double inv_dt, double *__restrict__ r) {
  __shared__ DgParams P;
  extern __shared__ double fs[];   // [3][p3][5] volume fluxes
  load_params(prm, &P);
  const int p = P.p, p3 = p * p * p, n = p - 1;
  const int e = blockIdx.x;
  const int node = threadIdx.x;
  const bool live = node < p3;
  T qn[5], gn[15];
  if (live) {
    const int64_t id = (int64_t)e * p3 + node;
    for (int v = 0; v < 5; ++v) qn[v] = at<T>(q, dq, id * 5 + v);
    for (int t = 0; t < 15; ++t) gn[t] = at<T>(g, dg, id * 15 + t);
    for (int d = 0; d < 3; ++d) {
      T fa[5], fv[5];
      flux_adv(qn, d, P.gamma, fa);
      flux_visc(qn, gn, d, P, fv);
      for (int v = 0; v < 5; ++v) fs[(d * p3 + node) * 5 + v] = part(fa[v] - fv[v]);
    }
  }
  __syncthreads();
  if (!live) return;
  const int c[3] = {node % p, (node / p) % p, node / (p * p)};
  double h[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int d = 0; d < 3; ++d) {
    const int l = c[d];
    double rd[5];
    for (int v = 0; v < 5; ++v) {
      double acc = 0.0;
      for (int a = 0; a < p; ++a) acc += P.vw[l][a] * fs[(d * p3 + node_with(node, p, d, a)) * 5 + v];
      rd[v] = acc;
    }
    if (l == n) {
      const int64_t nb = (int64_t)nbr_elem(e, P.k_elem, d, 1) * p3 + node_with(node, p, d, 0);
      T qb[5], gb[15], fh[5];
      for (int v = 0; v < 5; ++v) qb[v] = at<T>(q, dq, nb * 5 + v);
      if constexpr (SIPG) {
        T bn[15];
        for (int t = 0; t < 15; ++t) bn[t] = at<T>(gbq, dgb, ((int64_t)e * p3 + node) * 15 + t);
        for (int t = 0; t < 15; ++t) gb[t] = at<T>(gbq, dgb, nb * 15 + t);
        face_flux_sipg(qn, bn, qb, gb, d, P, fh);
      } else {
        for (int t = 0; t < 15; ++t) gb[t] = at<T>(g, dg, nb * 15 + t);
        face_flux(qn, gn, qb, gb, d, P, fh);
      }
      for (int v = 0; v < 5; ++v) rd[v] += part(fh[v]);
    }
    if (l == 0) {
      const int64_t nb = (int64_t)nbr_elem(e, P.k_elem, d, -1) * p3 + node_with(node, p, d, n);
      T qb[5], gb[15], fh[5];
      for (int v = 0; v < 5; ++v) qb[v] = at<T>(q, dq, nb * 5 + v);
      if constexpr (SIPG) {
        T bn[15];
        for (int t = 0; t < 15; ++t) bn[t] = at<T>(gbq, dgb, ((int64_t)e * p3 + node) * 15 + t);
        for (int t = 0; t < 15; ++t) gb[t] = at<T>(gbq, dgb, nb * 15 + t);
        face_flux_sipg(qb, gb, qn, bn, d, P, fh);
      } else {
        for (int t = 0; t < 15; ++t) gb[t] = at<T>(g, dg, nb * 15 + t);
        face_flux(qb, gb, qn, gn, d, P, fh);
      }
      for (int v = 0; v < 5; ++v) rd[v] -= part(fh[v]);
    }
    for (int v = 0; v < 5; ++v) h[v] += rd[v] / P.w[l];
  }
  const double m = P.jac * P.w[c[0]] * P.w[c[1]] * P.w[c[2]];
  const int64_t id = (int64_t)e * p3 + node;
  double *re = r + id * 5;
  for (int v = 0; v < 5; ++v) {
    double val = m * P.s * h[v];
    if constexpr (std::is_same<T, Dual>::value) {
      val += m * inv_dt * dq[id * 5 + v];
    } else {
      if (q_s) val += m * inv_dt * (qn[v] - q_s[id * 5 + v]);
    }
    re[v] = val;
  }
}

// The same operator in two parts, for the Newton-matrix product on dual
// numbers, where the fused kernel holds a node's state, gradient, its face
// neighbour's state and gradient and the flux temporaries at once and spills:
//   volume_kernel: r = M inv_dt dq + the volume sums (every node);
//   face_kernel (one launch per direction d): every +e_d face node pair
//     evaluates its numerical flux once and adds it to the node on the
//     minus side and subtracts it from the node on the plus side.
// Within one launch no two face pairs share a node; the launches follow each
// other on the stream.  Equal to residual_kernel up to the order of the sums.
template <class T>
__global__ __launch_bounds__(512) void volume_kernel(const DgParams *__restrict__ prm, const double *__restrict__ q,
                                                     const double *__restrict__ dq, const double *__restrict__ g,
                                                     const double *__restrict__ dg, const double *__restrict__ q_s,
                                                     double inv_dt, double *__restrict__ r) {
  __shared__ DgParams P;
  extern __shared__ double fs[];   // [3][p3][5] volume fluxes
  load_params(prm, &P);
  const int p = P.p, p3 = p * p * p;
  const int e = blockIdx.x;
  const int node = threadIdx.x;
  const bool live = node < p3;
  const int64_t id = (int64_t)e * p3 + node;
  if (live) {
    T qn[5], gn[15];
    for (int v = 0; v < 5; ++v) qn[v] = at<T>(q, dq, id * 5 + v);
    for (int t = 0; t < 15; ++t) gn[t] = at<T>(g, dg, id * 15 + t);
    for (int d = 0; d < 3; ++d) {
      T fa[5], fv[5];
      flux_adv(qn, d, P.gamma, fa);
      flux_visc(qn, gn, d, P, fv);
      for (int v = 0; v < 5; ++v) fs[(d * p3 + node) * 5 + v] = part(fa[v] - fv[v]);
    }
  }
  __syncthreads();
  if (!live) return;
  const int c[3] = {node % p, (node / p) % p, node / (p * p)};
  double h[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int d = 0; d < 3; ++d) {
    const int l = c[d];
    for (int v = 0; v < 5; ++v) {
      double acc = 0.0;
      for (int a = 0; a < p; ++a) acc += P.vw[l][a] * fs[(d * p3 + node_with(node, p, d, a)) * 5 + v];
      h[v] += acc / P.w[l];
    }
  }
  const double m = P.jac * P.w[c[0]] * P.w[c[1]] * P.w[c[2]];
  double *re = r + id * 5;
  for (int v = 0; v < 5; ++v) {
    double val = m * P.s * h[v];
    if constexpr (std::is_same<T, Dual>::value) {
      val += m * inv_dt * dq[id * 5 + v];
    } else {
      if (q_s) val += m * inv_dt * (q[id * 5 + v] - q_s[id * 5 + v]);
    }
    re[v] = val;
  }
}

template <class T, bool SIPG, int d>
__global__ __launch_bounds__(256) void face_kernel(const DgParams *__restrict__ prm, int64_t n_pairs,
                                                   const double *__restrict__ q, const double *__restrict__ dq,
                                                   const double *__restrict__ g, const double *__restrict__ dg,
                                                   const double *__restrict__ gbq, const double *__restrict__ dgb,
                                                   double *__restrict__ r) {
  __shared__ DgParams P;
  load_params(prm, &P);
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n_pairs) return;
  const int p = P.p, p2 = p * p, p3 = p2 * p, n = p - 1;
  const int e = (int)(idx / p2), tt = (int)(idx % p2), t1 = tt % p, t2 = tt / p;
  // transverse directions of d in increasing order take (t1, t2)
  int c[3];
  c[d] = n;
  c[d == 0 ? 1 : 0] = t1;
  c[d == 2 ? 1 : 2] = t2;
  const int node_l = c[0] + p * c[1] + p2 * c[2];
  const int node_r = node_with(node_l, p, d, 0);
  const int64_t il = (int64_t)e * p3 + node_l;
  const int64_t ir = (int64_t)nbr_elem(e, P.k_elem, d, 1) * p3 + node_r;
  // the flux term by term, one side's gradient live at a time (fewer registers
  // than face_flux / face_flux_sipg, the same terms)
  T ql[5], qr[5], fh[5];
  for (int v = 0; v < 5; ++v) {
    ql[v] = at<T>(q, dq, il * 5 + v);
    qr[v] = at<T>(q, dq, ir * 5 + v);
  }
  const double *gsrc = SIPG ? gbq : g, *dgsrc = SIPG ? dgb : dg;
  {
    T gs[15], fv[5];
    for (int t = 0; t < 15; ++t) gs[t] = at<T>(gsrc, dgsrc, il * 15 + t);
    flux_visc(ql, gs, d, P, fv);
    for (int v = 0; v < 5; ++v) fh[v] = -0.5 * fv[v];
  }
  {
    T gs[15], fv[5];
    for (int t = 0; t < 15; ++t) gs[t] = at<T>(gsrc, dgsrc, ir * 15 + t);
    flux_visc(qr, gs, d, P, fv);
    for (int v = 0; v < 5; ++v) fh[v] -= 0.5 * fv[v];
  }
  if constexpr (SIPG) {
    T qm[5], jg[15], fv[5];
    for (int t = 0; t < 15; ++t) jg[t] = 0.0;
    for (int v = 0; v < 5; ++v) {
      qm[v] = 0.5 * (ql[v] + qr[v]);
      jg[d * 5 + v] = qr[v] - ql[v];
    }
    flux_visc(qm, jg, d, P, fv);
    for (int v = 0; v < 5; ++v) fh[v] -= P.sigma * fv[v];
  }
  {
    T fa[5];
    flux_adv(ql, d, P.gamma, fa);
    for (int v = 0; v < 5; ++v) fh[v] += 0.5 * fa[v];
    flux_adv(qr, d, P.gamma, fa);
    for (int v = 0; v < 5; ++v) fh[v] += 0.5 * fa[v];
    const Prim<T> a = prim(ql, P.gamma), b = prim(qr, P.gamma);
    const T lam_l = vabs(a.u[d]) + vsqrt(P.gamma * a.p / a.rho);
    const T lam_r = vabs(b.u[d]) + vsqrt(P.gamma * b.p / b.rho);
    const T lam = lam_l >= lam_r ? lam_l : lam_r;
    for (int v = 0; v < 5; ++v) fh[v] -= 0.5 * lam * (qr[v] - ql[v]);
  }
  const double cf = P.jac * P.s * P.w[t1] * P.w[t2];
  for (int v = 0; v < 5; ++v) {
    const double f = cf * part(fh[v]);
    r[il * 5 + v] += f;
    r[ir * 5 + v] -= f;
  }
}

// Gauss-Lobatto nodes and weights (Newton on L_{N+1} - L_{N-1} from Chebyshev
// points) and the barycentric derivative matrix with the negative-sum diagonal.
void gl_operators(int nord, double *x, double *w, double d[kMaxP][kMaxP]) {
  const int p = nord + 1;
  auto leg = [](int k, double t, double &lk, double &dk) {
    double l0 = 1.0, l1 = t, d0 = 0.0, d1 = 1.0;
    if (k == 0) {
      lk = 1.0;
      dk = 0.0;
      return;
    }
    for (int m = 2; m <= k; ++m) {
      const double l2 = ((2 * m - 1) * t * l1 - (m - 1) * l0) / m;
      const double d2 = d0 + (2 * m - 1) * l1;
      l0 = l1;
      l1 = l2;
      d0 = d1;
      d1 = d2;
    }
    lk = l1;
    dk = d1;
  };
  for (int j = 0; j < p; ++j) x[j] = -std::cos(M_PI * j / nord);
  for (int j = 1; j < nord; ++j) {
    for (int it = 0; it < 100; ++it) {
      double lp, dp, lm, dm, ln, dn;
      leg(nord + 1, x[j], lp, dp);
      leg(nord - 1, x[j], lm, dm);
      leg(nord, x[j], ln, dn);
      const double step = (lp - lm) / ((2 * nord + 1) * ln);
      x[j] -= step;
      if (std::fabs(step) < 1e-16) break;
    }
  }
  x[0] = -1.0;
  x[nord] = 1.0;
  for (int j = 0; j < p; ++j) {
    double ln, dn;
    leg(nord, x[j], ln, dn);
    w[j] = 2.0 / (nord * (nord + 1) * ln * ln);
  }
  std::vector<double> lam(p, 1.0);
  for (int j = 0; j < p; ++j)
    for (int i = 0; i < p; ++i)
      if (i != j) lam[j] /= (x[j] - x[i]);
  for (int i = 0; i < p; ++i) {
    double sum = 0.0;
    for (int j = 0; j < p; ++j) {
      if (i == j) continue;
      d[i][j] = (lam[j] / lam[i]) / (x[i] - x[j]);
      sum += d[i][j];
    }
    d[i][i] = -sum;
  }
}

}  // namespace

// Metric terms of curved elements from the node positions xyz (3 doubles per
// node, natural node order), on the host: with X the element's coordinates
// relative to its first node, dX[j][m] = d X_m / d xi_j by the GL derivative
// matrix, and for (n, m, l) cyclic
//   (J a^i)_n = - e_i . curl_xi( X_l grad_xi X_m ),
// the conservative curl form, whose discrete divergence vanishes identically;
// J = det(dX).  out: 10 doubles per node, (J a^i)_n at 3 i + n, J at 9.
// Returns false if some J is not positive and finite.
bool curved_metrics(const DgParams &P, int64_t n_elem, const double *xyz, std::vector<double> &out) {
  const int p = P.p, p3 = p * p * p;
  out.assign((size_t)n_elem * p3 * 10, 0.0);
  std::vector<double> X((size_t)p3 * 3), dX((size_t)p3 * 9), V((size_t)p3 * 3);
  auto with = [&](int node, int d, int l) {
    int c[3] = {node % p, (node / p) % p, node / (p * p)};
    c[d] = l;
    return c[0] + p * c[1] + p * p * c[2];
  };
  auto deriv = [&](const std::vector<double> &f, int stride, int comp, int node, int d) {
    const int l = d == 0 ? node % p : d == 1 ? (node / p) % p : node / (p * p);
    double acc = 0.0;
    for (int a = 0; a < p; ++a) acc += P.d[l][a] * f[(size_t)with(node, d, a) * stride + comp];
    return acc;
  };
  for (int64_t e = 0; e < n_elem; ++e) {
    const double *xe = xyz + (size_t)e * p3 * 3;
    for (int t = 0; t < p3; ++t)
      for (int m = 0; m < 3; ++m) X[(size_t)t * 3 + m] = xe[t * 3 + m] - xe[m];
    for (int t = 0; t < p3; ++t)
      for (int j = 0; j < 3; ++j)
        for (int m = 0; m < 3; ++m) dX[(size_t)t * 9 + 3 * j + m] = deriv(X, 3, m, t, j);
    double *oe = out.data() + (size_t)e * p3 * 10;
    for (int nn = 0; nn < 3; ++nn) {
      const int m = (nn + 1) % 3, l = (nn + 2) % 3;
      for (int t = 0; t < p3; ++t)
        for (int j = 0; j < 3; ++j) V[(size_t)t * 3 + j] = X[(size_t)t * 3 + l] * dX[(size_t)t * 9 + 3 * j + m];
      for (int t = 0; t < p3; ++t)
        for (int i = 0; i < 3; ++i) {
          const int j = (i + 1) % 3, k = (i + 2) % 3;
          oe[(size_t)t * 10 + 3 * i + nn] = -(deriv(V, 3, k, t, j) - deriv(V, 3, j, t, k));
        }
    }
    for (int t = 0; t < p3; ++t) {
      const double *a = dX.data() + (size_t)t * 9;
      const double det = a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
                         a[2] * (a[3] * a[7] - a[4] * a[6]);
      if (!(det > 0.0) || !std::isfinite(det)) return false;
      oe[(size_t)t * 10 + 9] = det;
    }
  }
  return true;
}

// ---------------------------------------------------------------------------
// Element blocks of the backward-Euler Newton matrix A = M/dt + dH/dQ on the
// device (Sections 2.1.1 and 2.1.2: the linearised Lax-Friedrichs advective
// flux and the linearised BR1 viscous flux through the lifted gradient,
// eq. GradDGImp; eq. NewtonLinSys1).  Every 5x5 node block of dH/dQ is a
// linear combination of pointwise 5x5 Jacobians
//   Ja_d  = d f^a_d / d q,   Jv_d = d f^nu_d / d q (gradient held),
//   G_dd' = d f^nu_d / d g_d'  (g_d' the lifted gradient along d'),
//   PL_d, PR_d = d Fhat_d / d q^-, d q^+  (the advective face flux of a +d face),
// whose coefficients depend only on the mesh: the Gauss-Lobatto weights w,
// the derivative matrix D and the element size (s = 2/h).  With
//   c_t = J s w_t1 w_t2,  Vw[l][a] = -w_a D[a][l],
//   B[l][a] = Vw[l][a] + [l = a = N]/2 - [l = a = 0]/2,
//   L[b][a] = s (D[b][a] - [b = a = N]/(2 w_N) + [b = a = 0]/(2 w_0)),
// row (t, l) of direction d's line and column (t, a) of the same element get
//   c_t (Vw[l][a] Ja_d(a) - B[l][a] Jv_d(a) - sum_b B[l][b] L[b][a] G_dd(b)),
// the plane couplings get -c_(b,c) B[l][a] L[b][b'] G_dd'(a, b, c), and the
// face nodes pick up the face Jacobians and the lifting across the face
// (+-s/(2w) to the node across it).  The host writes that linear map once per
// order as a list of terms (destination node pair relative to the row's
// element, source Jacobian relative to the same element, coefficient); the
// device forms the pointwise Jacobians on dual numbers and sums the terms of
// every destination block into A_ii, A_ib, A_bi and the A_bb pattern.
// ---------------------------------------------------------------------------
constexpr int kPjNode = 15;   // node Jacobians: Ja_d at d, Jv_d at 3 + d, G_dd' at 6 + 3 d + d'

struct JacTerm {
  int32_t rn, col_off, cn, src_off, slot;   // slot -1: the mass term (identity times inv_dt)
  double coef;
};

// offsets (dx, dy, dz) in {-1, 0, 1}^3 as 0..26
static inline int off_code(int dx, int dy, int dz) { return (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1); }

// every term of dH/dQ + M/dt for elements of order N = p - 1 on Cartesian
// cubes (jac = (h/2)^3, s = 2/h) of a K^3 periodic mesh, merged and sorted by
// destination
std::vector<JacTerm> jac_terms(const DgParams &P) {
  const int p = P.p, n = p - 1;
  std::vector<JacTerm> t;
  double bh[kMaxP][kMaxP], lo[kMaxP][kMaxP];
  for (int l = 0; l < p; ++l)
    for (int a = 0; a < p; ++a) {
      bh[l][a] = -P.w[a] * P.d[a][l];
      lo[l][a] = P.s * P.d[l][a];
    }
  bh[n][n] += 0.5;
  bh[0][0] -= 0.5;
  lo[n][n] -= P.s / (2 * P.w[n]);
  lo[0][0] += P.s / (2 * P.w[0]);
  const double hi = P.s / (2 * P.w[n]), lw = -P.s / (2 * P.w[0]);
  auto node = [p](const int c[3]) { return c[0] + p * c[1] + p * p * c[2]; };
  auto unit = [](int d, int sg, int o[3]) {
    o[0] = o[1] = o[2] = 0;
    o[d] = sg;
  };
  // with two elements per direction the neighbours at -1 and +1 are one
  // element: column offsets are taken modulo 2 so that the terms of a block
  // reached both ways are summed into one destination (in a fixed order)
  const bool k2 = P.k_elem == 2;
  auto add = [&](int rn, const int co[3], int cn, const int so[3], int slot, double coef) {
    if (coef == 0.0) return;
    int c3[3] = {co[0], co[1], co[2]};
    if (k2)
      for (int ax = 0; ax < 3; ++ax) c3[ax] = c3[ax] < 0 ? 1 : c3[ax];
    t.push_back({rn, off_code(c3[0], c3[1], c3[2]), cn, off_code(so[0], so[1], so[2]), slot, coef});
  };
  const int Z[3] = {0, 0, 0};
  int up[3], dn[3], o2[3];
  for (int d = 0; d < 3; ++d) {
    const int t0a = d == 0 ? 1 : 0, t1a = d == 2 ? 1 : 2;   // transverse axes, ascending
    unit(d, 1, up);
    unit(d, -1, dn);
    for (int u0 = 0; u0 < p; ++u0)
      for (int u1 = 0; u1 < p; ++u1) {
        const double ct = P.jac * P.s * P.w[u0] * P.w[u1];
        auto nd = [&](int lin) {
          int c[3];
          c[d] = lin;
          c[t0a] = u0;
          c[t1a] = u1;
          return node(c);
        };
        const int face = p * p * p * kPjNode + (d * p * p + u1 * p + u0) * 2;   // PL; PR at +1 (higher axis first)
        for (int l = 0; l < p; ++l)
          for (int a = 0; a < p; ++a) {
            add(nd(l), Z, nd(a), Z, nd(a) * kPjNode + d, ct * P.vw[l][a]);
            add(nd(l), Z, nd(a), Z, nd(a) * kPjNode + 3 + d, -ct * bh[l][a]);
            for (int b = 0; b < p; ++b) add(nd(l), Z, nd(a), Z, nd(b) * kPjNode + 6 + 4 * d, -ct * bh[l][b] * lo[b][a]);
          }
        // own face terms: the face Jacobians and the neighbour's lifting across the face
        add(nd(n), Z, nd(n), Z, face, ct);
        add(nd(n), Z, nd(n), up, nd(0) * kPjNode + 6 + 4 * d, ct * P.s / (4 * P.w[0]));
        add(nd(0), Z, nd(0), dn, face + 1, -ct);
        add(nd(0), Z, nd(0), dn, nd(n) * kPjNode + 6 + 4 * d, ct * P.s / (4 * P.w[n]));
        // columns in the neighbours along d
        for (int l = 0; l < p; ++l) {
          add(nd(l), up, nd(0), Z, nd(n) * kPjNode + 6 + 4 * d, -bh[l][n] * ct * hi);
          add(nd(l), dn, nd(n), Z, nd(0) * kPjNode + 6 + 4 * d, -bh[l][0] * ct * lw);
        }
        add(nd(n), up, nd(0), Z, face + 1, ct);
        add(nd(n), up, nd(0), up, nd(0) * kPjNode + 3 + d, -0.5 * ct);
        add(nd(0), dn, nd(n), dn, face, -ct);
        add(nd(0), dn, nd(n), dn, nd(n) * kPjNode + 3 + d, 0.5 * ct);
        for (int a = 0; a < p; ++a) {
          add(nd(n), up, nd(a), up, nd(0) * kPjNode + 6 + 4 * d, -0.5 * ct * lo[0][a]);
          add(nd(0), dn, nd(a), dn, nd(n) * kPjNode + 6 + 4 * d, 0.5 * ct * lo[n][a]);
        }
      }
    for (int dp = 0; dp < 3; ++dp) {
      if (dp == d) continue;
      const int th = 3 - d - dp;
      auto nd3 = [&](int ad, int bdp, int ct_) {
        int c[3];
        c[d] = ad;
        c[dp] = bdp;
        c[th] = ct_;
        return node(c);
      };
      const int gs = 6 + 3 * d + dp;
      for (int b = 0; b < p; ++b)
        for (int c = 0; c < p; ++c) {
          const double ct = P.jac * P.s * P.w[b] * P.w[c];
          for (int l = 0; l < p; ++l)
            for (int a = 0; a < p; ++a)
              for (int bq = 0; bq < p; ++bq)
                add(nd3(l, b, c), Z, nd3(a, bq, c), Z, nd3(a, b, c) * kPjNode + gs, -ct * bh[l][a] * lo[b][bq]);
        }
      // lifting across a dp-face of the element itself
      for (int side = 0; side < 2; ++side) {
        const int b = side ? n : 0, nb = side ? 0 : n, sg = side ? 1 : -1;
        const double cf = side ? hi : lw;
        unit(dp, sg, o2);
        for (int c = 0; c < p; ++c) {
          const double ct = P.jac * P.s * P.w[b] * P.w[c];
          for (int l = 0; l < p; ++l)
            for (int a = 0; a < p; ++a)
              add(nd3(l, b, c), o2, nd3(a, nb, c), Z, nd3(a, b, c) * kPjNode + gs, -ct * cf * bh[l][a]);
        }
      }
      // the neighbour across the d-face: its plane couplings reach the face row
      for (int side = 0; side < 2; ++side) {
        const int lr = side ? n : 0, lm = side ? 0 : n, sd = side ? 1 : -1;
        const double sg = side ? 0.5 : -0.5;
        int on[3];
        unit(d, sd, on);
        for (int b = 0; b < p; ++b)
          for (int c = 0; c < p; ++c) {
            const double ct = P.jac * P.s * P.w[b] * P.w[c];
            for (int bq = 0; bq < p; ++bq)
              add(nd3(lr, b, c), on, nd3(lm, bq, c), on, nd3(lm, b, c) * kPjNode + gs, -sg * ct * lo[b][bq]);
          }
        for (int s2 = 0; s2 < 2; ++s2) {
          const int b = s2 ? n : 0, nb = s2 ? 0 : n, sg2 = s2 ? 1 : -1;
          const double cf = s2 ? hi : lw;
          int oc[3] = {on[0], on[1], on[2]};
          oc[dp] += sg2;
          for (int c = 0; c < p; ++c) {
            const double ct = P.jac * P.s * P.w[b] * P.w[c];
            add(nd3(lr, b, c), oc, nd3(lm, nb, c), on, nd3(lm, b, c) * kPjNode + gs, -sg * ct * cf);
          }
        }
      }
    }
  }
  // M / dt on the diagonal (the coefficient is the mass; inv_dt enters on the device)
  for (int k = 0; k < p; ++k)
    for (int j = 0; j < p; ++j)
      for (int i = 0; i < p; ++i) {
        const int c[3] = {i, j, k};
        add(node(c), Z, node(c), Z, -1, P.jac * P.w[i] * P.w[j] * P.w[k]);
      }
  std::sort(t.begin(), t.end(), [](const JacTerm &a, const JacTerm &b) {
    if (a.rn != b.rn) return a.rn < b.rn;
    if (a.col_off != b.col_off) return a.col_off < b.col_off;
    if (a.cn != b.cn) return a.cn < b.cn;
    if (a.src_off != b.src_off) return a.src_off < b.src_off;
    return a.slot < b.slot;
  });
  std::vector<JacTerm> m;
  for (const JacTerm &x : t) {
    if (!m.empty() && m.back().rn == x.rn && m.back().col_off == x.col_off && m.back().cn == x.cn &&
        m.back().src_off == x.src_off && m.back().slot == x.slot)
      m.back().coef += x.coef;
    else
      m.push_back(x);
  }
  return m;
}

// what the block assembly reads and writes (uniform order, periodic K^3 mesh)
struct JacBlocksArgs {
  const int4 *dest;            // [n_dest] (row node, column element offset, column node, first term)
  const int2 *term;            // [n_terms] (source element offset, source slot; -1: mass)
  const double *coef;          // [n_terms]
  int n_dest, n_terms;
  const double *pj;            // pointwise Jacobians, rec blocks of 25 per element
  int rec, k;
  const int32_t *iidx, *rank;  // [p^3] interior index / boundary rank of each local node (-1 if none)
  int ni, nc, ncn, nb;         // n_i, n_c (DOFs), |C_e| (nodes), boundary nodes per element
  const int32_t *c_node;       // [n_elem * ncn] coupling sets, sorted per element
  const int64_t *bb_rowptr;
  const int32_t *bb_col;
  double *aii, *aib, *abi, *bb_val;
  double inv_dt;
  int32_t *flag;               // set when a nonzero block has no place in the plan's structure
};

// the element at offset code oc from e on the periodic K^3 mesh
__device__ __forceinline__ int elem_at(int e, int k, int oc) {
  int c[3] = {e % k, (e / k) % k, e / (k * k)};
  c[0] = (c[0] + oc % 3 - 1 + k) % k;
  c[1] = (c[1] + (oc / 3) % 3 - 1 + k) % k;
  c[2] = (c[2] + oc / 9 - 1 + k) % k;
  return c[0] + k * c[1] + k * k * c[2];
}

// advective Lax-Friedrichs flux of a +e_d face (the viscous face terms enter
// the blocks through Jv and G)
template <class T>
__device__ void face_flux_adv(const T ql[5], const T qr[5], int d, const DgParams &P, T fh[5]) {
  T fl[5], fr[5];
  flux_adv(ql, d, P.gamma, fl);
  flux_adv(qr, d, P.gamma, fr);
  const Prim<T> a = prim(ql, P.gamma), b = prim(qr, P.gamma);
  const T lam_l = vabs(a.u[d]) + vsqrt(P.gamma * a.p / a.rho);
  const T lam_r = vabs(b.u[d]) + vsqrt(P.gamma * b.p / b.rho);
  const T lam = lam_l >= lam_r ? lam_l : lam_r;
  for (int v = 0; v < 5; ++v) fh[v] = 0.5 * (fl[v] + fr[v]) - 0.5 * lam * (qr[v] - ql[v]);
}

// node Jacobians: column kk of each 5x5 block from one dual evaluation seeded
// on input kk; block layout [row v][column kk]
__global__ __launch_bounds__(256) void pj_node_kernel(const DgParams *__restrict__ prm, const double *__restrict__ q,
                                                      const double *__restrict__ g, double *__restrict__ pj,
                                                      int64_t n_nodes, int rec) {
  __shared__ DgParams P;
  load_params(prm, &P);
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n_nodes) return;
  const int p3 = P.p * P.p * P.p;
  const int64_t e = i / p3;
  const int node = (int)(i % p3);
  double *out = pj + (e * rec + (int64_t)node * kPjNode) * 25;
  double qv[5], gv[15];
  for (int v = 0; v < 5; ++v) qv[v] = q[i * 5 + v];
  for (int t = 0; t < 15; ++t) gv[t] = g[i * 15 + t];
  for (int d = 0; d < 3; ++d) {
    for (int kk = 0; kk < 5; ++kk) {
      Dual qd[5], gd[15], f[5];
      for (int v = 0; v < 5; ++v) qd[v] = Dual(qv[v], v == kk ? 1.0 : 0.0);
      for (int t = 0; t < 15; ++t) gd[t] = Dual(gv[t], 0.0);
      flux_adv(qd, d, P.gamma, f);
      for (int v = 0; v < 5; ++v) out[d * 25 + v * 5 + kk] = f[v].d;
      flux_visc(qd, gd, d, P, f);
      for (int v = 0; v < 5; ++v) out[(3 + d) * 25 + v * 5 + kk] = f[v].d;
    }
    for (int dp = 0; dp < 3; ++dp)
      for (int kk = 0; kk < 5; ++kk) {
        Dual qd[5], gd[15], f[5];
        for (int v = 0; v < 5; ++v) qd[v] = Dual(qv[v], 0.0);
        for (int t = 0; t < 15; ++t) gd[t] = Dual(gv[t], t == dp * 5 + kk ? 1.0 : 0.0);
        flux_visc(qd, gd, d, P, f);
        for (int v = 0; v < 5; ++v) out[(6 + 3 * d + dp) * 25 + v * 5 + kk] = f[v].d;
      }
  }
}

// face Jacobians of every +e_d face of every element: thread (e, d, u1, u0),
// u0 / u1 the coordinates along the lower / higher transverse axis
__global__ __launch_bounds__(256) void pj_face_kernel(const DgParams *__restrict__ prm, const double *__restrict__ q,
                                                      double *__restrict__ pj, int64_t n_faces, int rec) {
  __shared__ DgParams P;
  load_params(prm, &P);
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n_faces) return;
  const int p = P.p, p2 = p * p, p3 = p2 * p, n = p - 1;
  const int64_t e = i / (3 * p2);
  const int r = (int)(i % (3 * p2));
  const int d = r / p2, u1 = (r % p2) / p, u0 = r % p;
  const int t0a = d == 0 ? 1 : 0, t1a = d == 2 ? 1 : 2;
  int c[3];
  c[t0a] = u0;
  c[t1a] = u1;
  c[d] = n;
  const int nl = c[0] + p * c[1] + p2 * c[2];
  c[d] = 0;
  const int nr = c[0] + p * c[1] + p2 * c[2];
  const int er = nbr_elem((int)e, P.k_elem, d, 1);
  double ql[5], qr[5];
  for (int v = 0; v < 5; ++v) {
    ql[v] = q[(e * p3 + nl) * 5 + v];
    qr[v] = q[((int64_t)er * p3 + nr) * 5 + v];
  }
  double *out = pj + (e * rec + (int64_t)p3 * kPjNode + r * 2) * 25;
  for (int side = 0; side < 2; ++side)
    for (int kk = 0; kk < 5; ++kk) {
      Dual a[5], b[5], f[5];
      for (int v = 0; v < 5; ++v) {
        a[v] = Dual(ql[v], side == 0 && v == kk ? 1.0 : 0.0);
        b[v] = Dual(qr[v], side == 1 && v == kk ? 1.0 : 0.0);
      }
      face_flux_adv(a, b, d, P, f);
      for (int v = 0; v < 5; ++v) out[side * 25 + v * 5 + kk] = f[v].d;
    }
}

// position of key in the sorted list a[0, len), or -1
__device__ __forceinline__ int find_sorted(const int32_t *__restrict__ a, int len, int32_t key) {
  int lo = 0, hi = len;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] < key)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo < len && a[lo] == key ? lo : -1;
}

// one thread per (element, destination block): the sum of its terms, written
// to A_ii, A_ib, A_bi or A_bb by the interior / boundary roles of its row and
// column nodes
__global__ __launch_bounds__(256) void jac_assemble_kernel(JacBlocksArgs a) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int e = blockIdx.y;
  if (t >= a.n_dest) return;
  const int4 ds = a.dest[t];
  const int tb = ds.w, te = t + 1 < a.n_dest ? a.dest[t + 1].w : a.n_terms;
  double acc[25];
#pragma unroll
  for (int u = 0; u < 25; ++u) acc[u] = 0.0;
  for (int j = tb; j < te; ++j) {
    const int2 ti = a.term[j];
    const double cf = a.coef[j];
    if (ti.y < 0) {
#pragma unroll
      for (int v = 0; v < 5; ++v) acc[v * 6] += cf * a.inv_dt;
      continue;
    }
    const double *__restrict__ src = a.pj + ((int64_t)elem_at(e, a.k, ti.x) * a.rec + ti.y) * 25;
#pragma unroll
    for (int u = 0; u < 25; ++u) acc[u] += cf * src[u];
  }
  bool nz = false;
#pragma unroll
  for (int u = 0; u < 25; ++u) nz = nz || acc[u] != 0.0;
  const int rn = ds.x, cn = ds.z;
  const int ce = elem_at(e, a.k, ds.y);
  const int ri = a.iidx[rn], ci = a.iidx[cn];
  double *dst = nullptr;
  int64_t ld = 0;
  if (ri >= 0 && ci >= 0) {
    if (ce == e) {
      ld = a.ni;
      dst = a.aii + (int64_t)e * a.ni * a.ni + (int64_t)(5 * ri) * ld + 5 * ci;
    }
  } else if (ri >= 0) {
    const int pos = find_sorted(a.c_node + (int64_t)e * a.ncn, a.ncn, ce * a.nb + a.rank[cn]);
    if (pos >= 0) {
      ld = a.nc;
      dst = a.aib + (int64_t)e * a.ni * a.nc + (int64_t)(5 * ri) * ld + 5 * pos;
    }
  } else if (ci >= 0) {
    const int pos = find_sorted(a.c_node + (int64_t)ce * a.ncn, a.ncn, e * a.nb + a.rank[rn]);
    if (pos >= 0) {
      ld = a.ni;
      dst = a.abi + (int64_t)ce * a.ni * a.nc + (int64_t)(5 * pos) * ld + 5 * ci;
    }
  } else {
    const int gr = e * a.nb + a.rank[rn], gc = ce * a.nb + a.rank[cn];
    const int64_t b0 = a.bb_rowptr[gr];
    const int pos = find_sorted(a.bb_col + b0, (int)(a.bb_rowptr[gr + 1] - b0), gc);
    if (pos >= 0) {
      ld = 5;
      dst = a.bb_val + (b0 + pos) * 25;
    }
  }
  if (!dst) {
    if (nz) a.flag[0] = 1;   // a nonzero block the plan's structure has no room for
    return;
  }
#pragma unroll
  for (int v = 0; v < 5; ++v)
#pragma unroll
    for (int w = 0; w < 5; ++w) dst[v * ld + w] = acc[v * 5 + w];
}

// structural check of a plan: one thread per (element, destination); flags a
// destination whose block has no place in the plan's coupling sets or A_bb
// pattern (the places are found as jac_assemble_kernel finds them)
__global__ __launch_bounds__(256) void jac_cover_kernel(JacBlocksArgs a) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int e = blockIdx.y;
  if (t >= a.n_dest) return;
  const int4 ds = a.dest[t];
  const int rn = ds.x, cn = ds.z;
  const int ce = elem_at(e, a.k, ds.y);
  const int ri = a.iidx[rn], ci = a.iidx[cn];
  bool found;
  if (ri >= 0 && ci >= 0)
    found = ce == e;
  else if (ri >= 0)
    found = find_sorted(a.c_node + (int64_t)e * a.ncn, a.ncn, ce * a.nb + a.rank[cn]) >= 0;
  else if (ci >= 0)
    found = find_sorted(a.c_node + (int64_t)ce * a.ncn, a.ncn, e * a.nb + a.rank[rn]) >= 0;
  else {
    const int gr = e * a.nb + a.rank[rn], gc = ce * a.nb + a.rank[cn];
    const int64_t b0 = a.bb_rowptr[gr];
    found = find_sorted(a.bb_col + b0, (int)(a.bb_rowptr[gr + 1] - b0), gc) >= 0;
  }
  if (!found) a.flag[0] = 1;
}

// x[0, n) = 0 in 16-byte stores (x 16-byte aligned), the odd last entry alone
__global__ void fill_zero_kernel(double *__restrict__ x, int64_t n) {
  double2 *x2 = reinterpret_cast<double2 *>(x);
  const int64_t n2 = n / 2;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n2; i += (int64_t)gridDim.x * blockDim.x)
    x2[i] = make_double2(0.0, 0.0);
  if (n % 2 && blockIdx.x == 0 && threadIdx.x == 0) x[n - 1] = 0.0;
}

struct DgContext {
  DgParams host;
  DgParams *dev = nullptr;
  double *g = nullptr;
  double *gd = nullptr;    // lifted gradient of a direction (allocated by the first Newton-matrix product)
  double *gb = nullptr;    // interior-penalty flux: broken gradient of the state (15 doubles per node)
  double *gbd = nullptr;   // ... and of a direction (with gd)
  double *met = nullptr;   // curved elements: 10 doubles per node (NULL: Cartesian cubes)
  uint64_t geo_gen = 0;    // bumped by every geometry change: captured graphs keyed on it recapture
  bool fused_residual = false;  // residual in one kernel (faces evaluated by both sides) instead of split
  int device = 0;          // the HIP device the object was created on
  int64_t n_nodes = 0;
  hipStream_t stream = nullptr;
  std::string last_error;
  // device Jacobian blocks: the term template of this order and the pointwise
  // Jacobians (allocated by the first scdg_dg_jacobian_blocks call)
  int jt_ndest = 0, jt_nterms = 0;
  int4 *jt_dest = nullptr;
  int2 *jt_term = nullptr;
  double *jt_coef = nullptr;
  int32_t *jt_iidx = nullptr, *jt_rank = nullptr, *jt_flag = nullptr;
  double *pj = nullptr;
  // the last plan checked for a place for every template block (uid, result)
  uint64_t cover_uid = 0;
  bool cover_ok = false;
};

}  // namespace scdg

using scdg::DgContext;

struct scdg_dg {
  DgContext c;
};

namespace scdg {

// The three face launches of the split operator (the direction is a template
// argument: the flux code indexes arrays by it).
template <class T>
hipError_t launch_faces(const DgContext &c, int n_elem, const double *q, const double *v, const double *gd,
                        const double *gbd, double *out, hipStream_t s) {
  const int64_t pairs = (int64_t)n_elem * c.host.p * c.host.p;
  const unsigned fgrid = (unsigned)((pairs + 255) / 256);
  if (c.host.sipg) {
    hipLaunchKernelGGL((face_kernel<T, true, 0>), dim3(fgrid), dim3(256), 0, s, c.dev, pairs, q, v, c.g, gd, c.gb,
                       gbd, out);
    hipLaunchKernelGGL((face_kernel<T, true, 1>), dim3(fgrid), dim3(256), 0, s, c.dev, pairs, q, v, c.g, gd, c.gb,
                       gbd, out);
    hipLaunchKernelGGL((face_kernel<T, true, 2>), dim3(fgrid), dim3(256), 0, s, c.dev, pairs, q, v, c.g, gd, c.gb,
                       gbd, out);
  } else {
    hipLaunchKernelGGL((face_kernel<T, false, 0>), dim3(fgrid), dim3(256), 0, s, c.dev, pairs, q, v, c.g, gd,
                       nullptr, nullptr, out);
    hipLaunchKernelGGL((face_kernel<T, false, 1>), dim3(fgrid), dim3(256), 0, s, c.dev, pairs, q, v, c.g, gd,
                       nullptr, nullptr, out);
    hipLaunchKernelGGL((face_kernel<T, false, 2>), dim3(fgrid), dim3(256), 0, s, c.dev, pairs, q, v, c.g, gd,
                       nullptr, nullptr, out);
  }
  return hipGetLastError();
}

hipError_t dg_residual_on(scdg_dg *dg, const double *q, const double *q_s, double inv_dt, double *r,
                          hipStream_t s) {
  auto &c = dg->c;
  const int p3 = c.host.p * c.host.p * c.host.p;
  const int n_elem = c.host.k_elem * c.host.k_elem * c.host.k_elem;
  const int threads = ((p3 + 63) / 64) * 64;
  if (c.met) {
    hipLaunchKernelGGL(lift_curved_kernel, dim3(n_elem), dim3(threads), sizeof(double) * 10 * p3, s, c.dev, q,
                       c.met, c.g);
    hipLaunchKernelGGL(residual_curved_kernel<double>, dim3(n_elem), dim3(threads), sizeof(double) * 15 * p3, s,
                       c.dev, q, nullptr, c.g, nullptr, c.met, q_s, inv_dt, r);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(lift_kernel, dim3(n_elem), dim3(threads), 0, s, c.dev, q, c.g, c.gb);
  if (c.fused_residual) {
    if (c.host.sipg)
      hipLaunchKernelGGL((residual_kernel<double, true>), dim3(n_elem), dim3(threads), sizeof(double) * 15 * p3, s,
                         c.dev, q, nullptr, c.g, nullptr, c.gb, nullptr, q_s, inv_dt, r);
    else
      hipLaunchKernelGGL((residual_kernel<double, false>), dim3(n_elem), dim3(threads), sizeof(double) * 15 * p3,
                         s, c.dev, q, nullptr, c.g, nullptr, nullptr, nullptr, q_s, inv_dt, r);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(volume_kernel<double>, dim3(n_elem), dim3(threads), sizeof(double) * 15 * p3, s, c.dev, q,
                     nullptr, c.g, nullptr, q_s, inv_dt, r);
  return launch_faces<double>(c, n_elem, q, nullptr, nullptr, nullptr, r, s);
}

// out = M inv_dt v + dH/dQ(q) v: the lifted gradients of q and of v (the
// lifting is linear), then the residual sums on dual numbers (value q,
// direction v).  c.gd must hold 15 doubles per node.
hipError_t dg_jacobian_apply_on(scdg_dg *dg, const double *q, const double *v, double inv_dt, double *out,
                                hipStream_t s, double *gd, double *gbd) {
  auto &c = dg->c;
  const int p3 = c.host.p * c.host.p * c.host.p;
  const int n_elem = c.host.k_elem * c.host.k_elem * c.host.k_elem;
  const int threads = ((p3 + 63) / 64) * 64;
  if (c.met) {
    hipLaunchKernelGGL(lift_curved_kernel, dim3(n_elem), dim3(threads), sizeof(double) * 10 * p3, s, c.dev, q,
                       c.met, c.g);
    hipLaunchKernelGGL(lift_curved_kernel, dim3(n_elem), dim3(threads), sizeof(double) * 10 * p3, s, c.dev, v,
                       c.met, gd);
    hipLaunchKernelGGL(residual_curved_kernel<Dual>, dim3(n_elem), dim3(threads), sizeof(double) * 15 * p3, s,
                       c.dev, q, v, c.g, gd, c.met, nullptr, inv_dt, out);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(lift_kernel, dim3(n_elem), dim3(threads), 0, s, c.dev, q, c.g, c.gb);
  hipLaunchKernelGGL(lift_kernel, dim3(n_elem), dim3(threads), 0, s, c.dev, v, gd, gbd);
  // volume sums, then the face fluxes once per face (see volume_kernel)
  hipLaunchKernelGGL(volume_kernel<Dual>, dim3(n_elem), dim3(threads), sizeof(double) * 15 * p3, s, c.dev, q, v,
                     c.g, gd, nullptr, inv_dt, out);
  return launch_faces<Dual>(c, n_elem, q, v, gd, gbd, out, s);
  return hipGetLastError();
}

int64_t dg_dof_count(const scdg_dg *dg) { return 5 * dg->c.n_nodes; }

// ---- allocation-free Newton-matrix product ----
// The direction's lifted gradient (15 doubles per node) of
// scdg_dg_jacobian_apply_noalloc lives in this file-scope device array, one copy
// per GPU, held until the process ends.  Its host-side name is not a device
// address: host code only ever uses the address hipGetSymbolAddress returns for
// the current device, kept per device in noalloc_ptr.
constexpr int64_t kNoAllocDoubles = SCDG_NOALLOC_SCRATCH_BYTES / sizeof(double);
static __device__ __align__(256) double scratch[kNoAllocDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex noalloc_mu;
double *noalloc_ptr[kMaxDevices] = {};
}  // namespace

// Resolve this device's copy of the scratch array; the caller has made `device`
// current.  Idempotent.
hipError_t noalloc_resolve(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(noalloc_mu);
  if (noalloc_ptr[device]) return hipSuccess;
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) return e != hipSuccess ? e : hipErrorInvalidSymbol;
  noalloc_ptr[device] = static_cast<double *>(ptr);
  return hipSuccess;
}

double *noalloc_lookup(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(noalloc_mu);
  return noalloc_ptr[device];
}

// What a captured residual launch depends on beyond the caller's vectors: the
// geometry generation (which kernels run, and on which metric buffer) and the
// object's own buffers.
void dg_graph_state(const scdg_dg *dg, uint64_t *gen, const void **g, const void **met, const void **params) {
  *gen = dg->c.geo_gen;
  *g = dg->c.g;
  *met = dg->c.met;
  *params = dg->c.dev;
}

std::string dg_last_error(const scdg_dg *dg) { return dg->c.last_error; }

bool dg_jacobian_shape(const scdg_dg *dg, int *k_elem, int *order, bool *cartesian_br1) {
  *k_elem = dg->c.host.k_elem;
  *order = dg->c.host.p - 1;
  *cartesian_br1 = !dg->c.met && !dg->c.host.sipg;
  return true;
}

scdg_status dg_jacobian_blocks_on(scdg_dg *dg, const JacPlanView &v, const double *q, double inv_dt, double *aii,
                                  double *aib, double *abi, double *bb_val) {
  auto &c = dg->c;
  const int p = c.host.p, p3 = p * p * p, n = p - 1;
  const int n_elem = c.host.k_elem * c.host.k_elem * c.host.k_elem;
  const int rec = p3 * kPjNode + 3 * p * p * 2;
  auto fail = [&](const char *what) {
    c.last_error = std::string("scdg_dg_jacobian_blocks: ") + what;
    return SCDG_ERR_HIP;
  };
  if (!c.jt_dest) {
    const std::vector<JacTerm> t = jac_terms(c.host);
    std::vector<int4> dest;
    std::vector<int2> term(t.size());
    std::vector<double> coef(t.size());
    for (size_t j = 0; j < t.size(); ++j) {
      if (j == 0 || t[j].rn != t[j - 1].rn || t[j].col_off != t[j - 1].col_off || t[j].cn != t[j - 1].cn)
        dest.push_back(make_int4(t[j].rn, t[j].col_off, t[j].cn, (int)j));
      term[j] = make_int2(t[j].src_off, t[j].slot);
      coef[j] = t[j].coef;
    }
    std::vector<int32_t> iidx(p3, -1), rank(p3, -1);
    int ni = 0, nb = 0;
    for (int node = 0; node < p3; ++node) {
      const int cc[3] = {node % p, (node / p) % p, node / (p * p)};
      const bool in = cc[0] >= 1 && cc[0] <= n - 1 && cc[1] >= 1 && cc[1] <= n - 1 && cc[2] >= 1 && cc[2] <= n - 1;
      if (in)
        iidx[node] = ni++;
      else
        rank[node] = nb++;
    }
    c.jt_ndest = (int)dest.size();
    c.jt_nterms = (int)t.size();
    if (hipMalloc(&c.jt_dest, sizeof(int4) * dest.size()) != hipSuccess ||
        hipMalloc(&c.jt_term, sizeof(int2) * term.size()) != hipSuccess ||
        hipMalloc(&c.jt_coef, sizeof(double) * coef.size()) != hipSuccess ||
        hipMalloc(&c.jt_iidx, sizeof(int32_t) * p3) != hipSuccess ||
        hipMalloc(&c.jt_rank, sizeof(int32_t) * p3) != hipSuccess ||
        hipMalloc(&c.jt_flag, sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&c.pj, sizeof(double) * 25 * (size_t)rec * n_elem) != hipSuccess)
      return SCDG_ERR_NOMEM;
    if (hipMemcpy(c.jt_dest, dest.data(), sizeof(int4) * dest.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c.jt_term, term.data(), sizeof(int2) * term.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c.jt_coef, coef.data(), sizeof(double) * coef.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c.jt_iidx, iidx.data(), sizeof(int32_t) * p3, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c.jt_rank, rank.data(), sizeof(int32_t) * p3, hipMemcpyHostToDevice) != hipSuccess)
      return fail("upload of the term template");
  }
  const hipStream_t s = c.stream;
  const int64_t n_ii = (int64_t)n_elem * v.ni * v.ni, n_ib = (int64_t)n_elem * v.ni * v.nc;
  const unsigned fill_grid = 8192;
  hipLaunchKernelGGL(fill_zero_kernel, dim3(fill_grid), dim3(256), 0, s, aii, n_ii);
  hipLaunchKernelGGL(fill_zero_kernel, dim3(fill_grid), dim3(256), 0, s, aib, n_ib);
  hipLaunchKernelGGL(fill_zero_kernel, dim3(fill_grid), dim3(256), 0, s, abi, n_ib);
  hipLaunchKernelGGL(fill_zero_kernel, dim3(fill_grid), dim3(256), 0, s, bb_val, v.nnzb * 25);
  if (hipMemsetAsync(c.jt_flag, 0, sizeof(int32_t), s) != hipSuccess) return fail("flag reset");
  const int threads = ((p3 + 63) / 64) * 64;
  hipLaunchKernelGGL(lift_kernel, dim3(n_elem), dim3(threads), 0, s, c.dev, q, c.g, nullptr);
  const int64_t n_nodes = (int64_t)n_elem * p3, n_faces = (int64_t)n_elem * 3 * p * p;
  hipLaunchKernelGGL(pj_node_kernel, dim3((unsigned)((n_nodes + 255) / 256)), dim3(256), 0, s, c.dev, q, c.g, c.pj,
                     n_nodes, rec);
  hipLaunchKernelGGL(pj_face_kernel, dim3((unsigned)((n_faces + 255) / 256)), dim3(256), 0, s, c.dev, q, c.pj,
                     n_faces, rec);
  JacBlocksArgs a;
  a.dest = c.jt_dest;
  a.term = c.jt_term;
  a.coef = c.jt_coef;
  a.n_dest = c.jt_ndest;
  a.n_terms = c.jt_nterms;
  a.pj = c.pj;
  a.rec = rec;
  a.k = c.host.k_elem;
  a.iidx = c.jt_iidx;
  a.rank = c.jt_rank;
  a.ni = v.ni;
  a.nc = v.nc;
  a.ncn = v.ncn;
  a.nb = v.nb;
  a.c_node = v.c_node;
  a.bb_rowptr = v.bb_rowptr;
  a.bb_col = v.bb_col;
  a.aii = aii;
  a.aib = aib;
  a.abi = abi;
  a.bb_val = bb_val;
  a.inv_dt = inv_dt;
  a.flag = c.jt_flag;
  const dim3 dest_grid((unsigned)((c.jt_ndest + 255) / 256), (unsigned)n_elem);
  if (c.cover_uid != v.plan_uid) {
    // does the plan hold a place for every block of the template?  (once per
    // plan; its coupling sets and A_bb pattern never change)
    c.cover_uid = 0;
    hipLaunchKernelGGL(jac_cover_kernel, dest_grid, dim3(256), 0, s, a);
    int32_t missing = 0;
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(&missing, c.jt_flag, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return fail("structure check");
    c.cover_uid = v.plan_uid;
    c.cover_ok = missing == 0;
    if (hipMemsetAsync(c.jt_flag, 0, sizeof(int32_t), s) != hipSuccess) return fail("flag reset");
  }
  hipLaunchKernelGGL(jac_assemble_kernel, dest_grid, dim3(256), 0, s, a);
  if (hipGetLastError() != hipSuccess) return fail("launch");
  // every block has a place: nothing to check, the call returns without waiting
  if (c.cover_ok) return SCDG_OK;
  int32_t flag = 0;
  if (hipMemcpyAsync(&flag, c.jt_flag, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail("synchronisation");
  if (flag) {
    c.last_error = "scdg_dg_jacobian_blocks: a nonzero block has no place in the plan's coupling sets or A_bb pattern";
    return SCDG_ERR_ARG;
  }
  return SCDG_OK;
}

}  // namespace scdg

extern "C" {

scdg_status scdg_dg_create(scdg_dg **out, const scdg_dg_params *prm, void *hip_stream) {
  if (!out || !prm || prm->k_elem < 2 || prm->order < 2 || prm->order > scdg::kMaxOrder ||
      prm->length <= 0 || prm->mach <= 0 || prm->reynolds <= 0 ||
      (prm->viscous_flux != SCDG_VISCOUS_BR1 && prm->viscous_flux != SCDG_VISCOUS_SIPG) ||
      !(prm->sipg_eta >= 0.0) || !std::isfinite(prm->sipg_eta))
    return SCDG_ERR_ARG;
  scdg_dg *dg = new (std::nothrow) scdg_dg();
  if (!dg) return SCDG_ERR_NOMEM;
  auto &c = dg->c;
  auto &P = c.host;
  P.k_elem = prm->k_elem;
  P.p = prm->order + 1;
  const double h = prm->length / prm->k_elem;
  P.s = 2.0 / h;
  P.jac = (h / 2) * (h / 2) * (h / 2);
  P.gamma = prm->gamma > 0 ? prm->gamma : 1.4;
  P.mach2 = prm->mach * prm->mach;
  P.inv_re = 1.0 / prm->reynolds;
  P.prandtl = prm->prandtl > 0 ? prm->prandtl : 0.72;
  P.suth = prm->sutherland_ratio > 0 ? prm->sutherland_ratio : 110.4 / 288.15;
  P.sipg = prm->viscous_flux == SCDG_VISCOUS_SIPG ? 1 : 0;
  P.sigma = (prm->sipg_eta > 0 ? prm->sipg_eta : 1.0) * (prm->order + 1) * (prm->order + 1) / h;
  double x[scdg::kMaxP];
  scdg::gl_operators(prm->order, x, P.w, P.d);
  for (int l = 0; l < P.p; ++l)
    for (int a = 0; a < P.p; ++a) P.vw[l][a] = -P.w[a] * P.d[a][l];
  c.stream = static_cast<hipStream_t>(hip_stream);
  c.n_nodes = (int64_t)prm->k_elem * prm->k_elem * prm->k_elem * P.p * P.p * P.p;
  if (hipGetDevice(&c.device) != hipSuccess) {
    delete dg;
    return SCDG_ERR_HIP;
  }
  // set-up of the allocation-free product: this device's scratch address (no
  // allocation; a failure is reported by scdg_dg_jacobian_apply_noalloc)
  (void)scdg::noalloc_resolve(c.device);
  if (hipMalloc(&c.dev, sizeof(scdg::DgParams)) != hipSuccess ||
      hipMalloc(&c.g, sizeof(double) * 15 * c.n_nodes) != hipSuccess ||
      (P.sipg && hipMalloc(&c.gb, sizeof(double) * 15 * c.n_nodes) != hipSuccess) ||
      hipMemcpy(c.dev, &P, sizeof(scdg::DgParams), hipMemcpyHostToDevice) != hipSuccess) {
    if (c.dev) (void)hipFree(c.dev);
    if (c.g) (void)hipFree(c.g);
    if (c.gb) (void)hipFree(c.gb);
    delete dg;
    return SCDG_ERR_NOMEM;
  }
  *out = dg;
  return SCDG_OK;
}

scdg_status scdg_dg_destroy(scdg_dg *dg) {
  if (!dg) return SCDG_OK;
  (void)hipStreamSynchronize(dg->c.stream);
  if (dg->c.dev) (void)hipFree(dg->c.dev);
  if (dg->c.g) (void)hipFree(dg->c.g);
  if (dg->c.gd) (void)hipFree(dg->c.gd);
  if (dg->c.gb) (void)hipFree(dg->c.gb);
  if (dg->c.gbd) (void)hipFree(dg->c.gbd);
  if (dg->c.met) (void)hipFree(dg->c.met);
  for (void *ptr : {(void *)dg->c.jt_dest, (void *)dg->c.jt_term, (void *)dg->c.jt_coef, (void *)dg->c.jt_iidx,
                    (void *)dg->c.jt_rank, (void *)dg->c.jt_flag, (void *)dg->c.pj})
    if (ptr) (void)hipFree(ptr);
  delete dg;
  return SCDG_OK;
}

scdg_status scdg_dg_residual(scdg_dg *dg, const double *q, const double *q_s, double inv_dt,
                             double *r) {
  if (!dg || !q || !r) return SCDG_ERR_ARG;
  return scdg::dg_residual_on(dg, q, q_s, inv_dt, r, dg->c.stream) == hipSuccess ? SCDG_OK : SCDG_ERR_HIP;
}

scdg_status scdg_dg_jacobian_apply(scdg_dg *dg, const double *q, const double *v, double inv_dt, double *out) {
  if (!dg || !q || !v || !out || !(inv_dt >= 0.0) || !std::isfinite(inv_dt)) return SCDG_ERR_ARG;
  auto &c = dg->c;
  if (!c.gd && hipMalloc(&c.gd, sizeof(double) * 15 * c.n_nodes) != hipSuccess) {
    c.gd = nullptr;
    return SCDG_ERR_NOMEM;
  }
  if (c.host.sipg && !c.gbd && hipMalloc(&c.gbd, sizeof(double) * 15 * c.n_nodes) != hipSuccess) {
    c.gbd = nullptr;
    return SCDG_ERR_NOMEM;
  }
  return scdg::dg_jacobian_apply_on(dg, q, v, inv_dt, out, c.stream, c.gd, c.gbd) == hipSuccess ? SCDG_OK
                                                                                                : SCDG_ERR_HIP;
}

scdg_status scdg_dg_jacobian_apply_noalloc(scdg_dg *dg, const double *q, const double *v, double inv_dt,
                                           double *out) {
  if (!dg || !q || !v || !out || !(inv_dt >= 0.0) || !std::isfinite(inv_dt)) return SCDG_ERR_ARG;
  auto &c = dg->c;
  if (c.host.sipg) {
    c.last_error = "scdg_dg_jacobian_apply_noalloc: Bassi-Rebay 1 flux only";
    return SCDG_ERR_UNSUPPORTED;
  }
  if (15 * c.n_nodes > scdg::kNoAllocDoubles) {
    c.last_error = "scdg_dg_jacobian_apply_noalloc: the mesh needs " + std::to_string(15 * 8 * c.n_nodes) +
                   " bytes of gradient scratch, above the fixed " +
                   std::to_string((long long)SCDG_NOALLOC_SCRATCH_BYTES) + "-byte array";
    return SCDG_ERR_UNSUPPORTED;
  }
  double *gd = scdg::noalloc_lookup(c.device);
  if (!gd) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != c.device || scdg::noalloc_resolve(c.device) != hipSuccess ||
        !(gd = scdg::noalloc_lookup(c.device))) {
      c.last_error = "scdg_dg_jacobian_apply_noalloc: no address for the scratch array on this device";
      return SCDG_ERR_HIP;
    }
  }
  return scdg::dg_jacobian_apply_on(dg, q, v, inv_dt, out, c.stream, gd, nullptr) == hipSuccess ? SCDG_OK
                                                                                              : SCDG_ERR_HIP;
}

scdg_status scdg_dg_set_geometry(scdg_dg *dg, const double *xyz) {
  if (!dg) return SCDG_ERR_ARG;
  auto &c = dg->c;
  if (hipStreamSynchronize(c.stream) != hipSuccess) return SCDG_ERR_HIP;
  if (!xyz) {
    if (c.met) (void)hipFree(c.met);
    c.met = nullptr;
    ++c.geo_gen;
    return SCDG_OK;
  }
  if (c.host.sipg) {
    c.last_error = "curved elements with the interior-penalty flux are not supported";
    return SCDG_ERR_UNSUPPORTED;
  }
  const int64_t n_elem = (int64_t)c.host.k_elem * c.host.k_elem * c.host.k_elem;
  std::vector<double> met;
  if (!scdg::curved_metrics(c.host, n_elem, xyz, met)) {
    c.last_error = "node positions give a non-positive or non-finite Jacobian";
    return SCDG_ERR_ARG;
  }
  ++c.geo_gen;
  if (!c.met && hipMalloc(&c.met, sizeof(double) * met.size()) != hipSuccess) {
    c.met = nullptr;
    return SCDG_ERR_NOMEM;
  }
  if (hipMemcpy(c.met, met.data(), sizeof(double) * met.size(), hipMemcpyHostToDevice) != hipSuccess)
    return SCDG_ERR_HIP;
  return SCDG_OK;
}

scdg_status scdg_dg_gradient(scdg_dg *dg, double *g_out) {
  if (!dg || !g_out) return SCDG_ERR_ARG;
  auto &c = dg->c;
  if (hipMemcpyAsync(g_out, c.g, sizeof(double) * 15 * c.n_nodes, hipMemcpyDeviceToDevice,
                     c.stream) != hipSuccess)
    return SCDG_ERR_HIP;
  return SCDG_OK;
}

}  // extern "C"
