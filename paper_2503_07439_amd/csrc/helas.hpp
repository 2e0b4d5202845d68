// Device helicity-amplitude routines for one event per lane, templated on the
// arithmetic type T (double or float).
//
// The paper's Born and real-emission amplitudes are sums of tree Feynman
// diagrams; these routines evaluate their building blocks: external spinors
// and polarisation vectors, off-shell currents at the fermion-fermion-vector,
// three-vector and four-vector vertices, and propagators.  Spinors use the
// chiral Dirac representation; vectors are stored with upper indices; the
// metric is (+,-,-,-).
//
// Every routine is phase- and coupling-free: the factors of i and the coupling
// constants of the Feynman rules are folded by the generator into the colour
// coefficients and into one overall factor applied in FP64.
//   fermion propagator  (pslash + m) / (p^2 - m^2)   [times i]
//   vector propagator   1 / p^2                      [times -i]
//   FFV vertex          gamma^mu                     [times i g  or  -i e Q]
//   VVV vertex          V_{mu nu rho}(k1, k2, k3)    [times g f^{abc}]
//   VVVV vertex         (g g - g g) per colour pair  [times -i g^2 f f]
#pragma once
#include <hip/hip_runtime.h>

#define NLO_HD __host__ __device__ __forceinline__

namespace nlo {

template <class T> struct cx { T r, i; };

// packed pairs of half-width floats (one event in each half of a register)
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

template <class T> struct w4 { cx<T> c[4]; };      // spinor, or vector with upper index

// exact values of up to two pairwise invariants 2 q_a.q_b (legs a < b, all
// momenta incoming) that replace the ones a prologue forms from the momenta;
// a0 < 0: none
struct PairOv {
  int a0 = -1, b0 = -1, a1 = -1, b1 = -1;
  double v0 = 0.0, v1 = 0.0;
};
template <class T> struct r4 { T v[4]; };          // real four-momentum

template <class T> NLO_HD cx<T> operator+(cx<T> a, cx<T> b) { return {a.r + b.r, a.i + b.i}; }
template <class T> NLO_HD cx<T> operator-(cx<T> a, cx<T> b) { return {a.r - b.r, a.i - b.i}; }
template <class T> NLO_HD cx<T> operator-(cx<T> a) { return {-a.r, -a.i}; }
template <class T> NLO_HD cx<T> operator*(cx<T> a, cx<T> b) {
  return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r};
}
template <class T> NLO_HD cx<T> operator*(T s, cx<T> a) { return {s * a.r, s * a.i}; }
template <class T> NLO_HD cx<T> mul_i(cx<T> a) { return {-a.i, a.r}; }
template <class T> NLO_HD cx<T> conj(cx<T> a) { return {a.r, -a.i}; }
template <class T> NLO_HD cx<T> czero() { return {T(0), T(0)}; }

template <class T> NLO_HD w4<T> operator+(const w4<T>& a, const w4<T>& b) {
  return {{a.c[0] + b.c[0], a.c[1] + b.c[1], a.c[2] + b.c[2], a.c[3] + b.c[3]}};
}
template <class T> NLO_HD w4<T> operator-(const w4<T>& a, const w4<T>& b) {
  return {{a.c[0] - b.c[0], a.c[1] - b.c[1], a.c[2] - b.c[2], a.c[3] - b.c[3]}};
}
template <class T> NLO_HD w4<T> operator*(cx<T> s, const w4<T>& a) {
  return {{s * a.c[0], s * a.c[1], s * a.c[2], s * a.c[3]}};
}
template <class T> NLO_HD w4<T> operator*(T s, const w4<T>& a) {
  return {{s * a.c[0], s * a.c[1], s * a.c[2], s * a.c[3]}};
}

// Minkowski products
template <class T> NLO_HD cx<T> mdot(const w4<T>& a, const w4<T>& b) {
  return a.c[0] * b.c[0] - a.c[1] * b.c[1] - a.c[2] * b.c[2] - a.c[3] * b.c[3];
}
template <class T> NLO_HD cx<T> mdot(const w4<T>& a, const r4<T>& p) {
  return p.v[0] * a.c[0] - p.v[1] * a.c[1] - p.v[2] * a.c[2] - p.v[3] * a.c[3];
}
// plain sum_k a_k b_k (row spinor times column spinor)
template <class T> NLO_HD cx<T> rdot(const w4<T>& a, const w4<T>& b) {
  return a.c[0] * b.c[0] + a.c[1] * b.c[1] + a.c[2] * b.c[2] + a.c[3] * b.c[3];
}

// ---------------------------------------------------------------------------
// slashed vectors in the chiral representation:
//   Vslash = [[0, V.sigma], [V.sigmabar, 0]],
//   V.sigma = [[V0-V3, -(V1-iV2)], [-(V1+iV2), V0+V3]],
//   V.sigmabar = [[V0+V3, V1-iV2], [V1+iV2, V0-V3]]
// ---------------------------------------------------------------------------
template <class T> NLO_HD w4<T> slash_col(const w4<T>& V, const w4<T>& c) {   // Vslash * column
  cx<T> vp = V.c[0] + V.c[3], vm = V.c[0] - V.c[3];
  cx<T> tp = V.c[1] + mul_i(V.c[2]), tm = V.c[1] - mul_i(V.c[2]);
  return {{vm * c.c[2] - tm * c.c[3], vp * c.c[3] - tp * c.c[2],
           vp * c.c[0] + tm * c.c[1], tp * c.c[0] + vm * c.c[1]}};
}
template <class T> NLO_HD w4<T> row_slash(const w4<T>& r, const w4<T>& V) {   // row * Vslash
  cx<T> vp = V.c[0] + V.c[3], vm = V.c[0] - V.c[3];
  cx<T> tp = V.c[1] + mul_i(V.c[2]), tm = V.c[1] - mul_i(V.c[2]);
  return {{r.c[2] * vp + r.c[3] * tp, r.c[2] * tm + r.c[3] * vm,
           r.c[0] * vm - r.c[1] * tp, r.c[1] * vp - r.c[0] * tm}};
}
template <class T> NLO_HD w4<T> pslash_col(const r4<T>& P, const w4<T>& c) {   // Pslash * column, P real
  T pp = P.v[0] + P.v[3], pm = P.v[0] - P.v[3];
  cx<T> tp = {P.v[1], P.v[2]}, tm = {P.v[1], -P.v[2]};
  return {{pm * c.c[2] - tm * c.c[3], pp * c.c[3] - tp * c.c[2],
           pp * c.c[0] + tm * c.c[1], tp * c.c[0] + pm * c.c[1]}};
}
template <class T> NLO_HD w4<T> row_pslash(const w4<T>& r, const r4<T>& P) {   // row * Pslash, P real
  T pp = P.v[0] + P.v[3], pm = P.v[0] - P.v[3];
  cx<T> tp = {P.v[1], P.v[2]}, tm = {P.v[1], -P.v[2]};
  return {{pp * r.c[2] + r.c[3] * tp, r.c[2] * tm + pm * r.c[3],
           pm * r.c[0] - r.c[1] * tp, pp * r.c[1] - r.c[0] * tm}};
}

// ---------------------------------------------------------------------------
// external states
// ---------------------------------------------------------------------------
// Fermion leg: chi+ = (a, b) is the helicity +1/2 eigenstate of sigma.phat,
// chi- = (-conj(b), a); wp = sqrt(E+|p|), wm = sqrt(E-|p|) (exactly 0 if massless).
template <class T> struct ferm_data { T a, br, bi, wp, wm; };
// Massless vector leg: e1 = eps1/sqrt2, e2 = eps2/sqrt2 (eps1 has no time
// component, eps2 has no time or z component).
template <class T> struct vec_data { T e1x, e1y, e1z, e2x, e2y; };

// u(p, lam) = (sqrt(E - lam|p|) chi_lam, sqrt(E + lam|p|) chi_lam)
template <class T> NLO_HD w4<T> wf_u(const ferm_data<T>& d, bool plus) {
  cx<T> x0 = plus ? cx<T>{d.a, T(0)} : cx<T>{-d.br, d.bi};
  cx<T> x1 = plus ? cx<T>{d.br, d.bi} : cx<T>{d.a, T(0)};
  T lo = plus ? d.wm : d.wp, hi = plus ? d.wp : d.wm;
  return {{lo * x0, lo * x1, hi * x0, hi * x1}};
}
// v(p, lam) = (-lam sqrt(E + lam|p|) chi_{-lam}, lam sqrt(E - lam|p|) chi_{-lam})
template <class T> NLO_HD w4<T> wf_v(const ferm_data<T>& d, bool plus) {
  cx<T> x0 = plus ? cx<T>{-d.br, d.bi} : cx<T>{d.a, T(0)};
  cx<T> x1 = plus ? cx<T>{d.a, T(0)} : cx<T>{d.br, d.bi};
  T f = plus ? -d.wp : d.wm, s = plus ? d.wm : -d.wp;
  return {{f * x0, f * x1, s * x0, s * x1}};
}
// row spinor psibar = psi^dagger gamma^0
template <class T> NLO_HD w4<T> wf_bar(const w4<T>& s) {
  return {{conj(s.c[2]), conj(s.c[3]), conj(s.c[0]), conj(s.c[1])}};
}
// eps(k, lam) = (-lam eps1 - i eps2)/sqrt2 for an incoming vector, its
// complex conjugate for an outgoing one
template <class T> NLO_HD w4<T> wf_eps(const vec_data<T>& d, bool plus, bool outgoing) {
  T l = plus ? T(-1) : T(1);
  T s = outgoing ? T(1) : T(-1);
  return {{cx<T>{T(0), T(0)}, cx<T>{l * d.e1x, s * d.e2x}, cx<T>{l * d.e1y, s * d.e2y}, cx<T>{l * d.e1z, T(0)}}};
}
// Real linear polarisations eps1 (k = 0) and eps2 (k = 1).  The helicity
// states are a unitary combination of them, so the sum of |A|^2 over the two
// helicities of a leg equals the sum over eps1 and eps2; the amplitudes with
// a real vector are cheaper.
template <class T> NLO_HD w4<T> wf_lin(const vec_data<T>& d, int k) {
  const T r2 = T(1.4142135623730951);
  return k == 0 ? w4<T>{{cx<T>{T(0), T(0)}, cx<T>{r2 * d.e1x, T(0)}, cx<T>{r2 * d.e1y, T(0)}, cx<T>{r2 * d.e1z, T(0)}}}
                : w4<T>{{cx<T>{T(0), T(0)}, cx<T>{r2 * d.e2x, T(0)}, cx<T>{r2 * d.e2y, T(0)}, cx<T>{T(0), T(0)}}};
}

// ---------------------------------------------------------------------------
// vertices and propagators
// ---------------------------------------------------------------------------
// column current through an FFV vertex: (Pslash + m) Vslash C / (P^2 - m^2)
template <class T> NLO_HD w4<T> ffv_col(const w4<T>& C, const w4<T>& V, const r4<T>& P, T den, T m) {
  w4<T> x = slash_col(V, C);
  w4<T> y = pslash_col(P, x);
  return den * (y + m * x);
}
// row current through an FFV vertex: R Vslash (-Pslash + m) / (P^2 - m^2)
template <class T> NLO_HD w4<T> ffv_row(const w4<T>& R, const w4<T>& V, const r4<T>& P, T den, T m) {
  w4<T> x = row_slash(R, V);
  w4<T> y = row_pslash(x, P);
  return den * (m * x - y);
}
// massless-fermion versions (no mass term)
template <class T> NLO_HD w4<T> ffv_col0(const w4<T>& C, const w4<T>& V, const r4<T>& P, T den) {
  return den * pslash_col(P, slash_col(V, C));
}
template <class T> NLO_HD w4<T> ffv_row0(const w4<T>& R, const w4<T>& V, const r4<T>& P, T den) {
  return (-den) * row_pslash(row_slash(R, V), P);
}
// fermion-pair current R gamma^nu C (no propagator); R Vslash C equals
// mdot(ffv_cur(R, C), V)
template <class T> NLO_HD w4<T> ffv_cur(const w4<T>& R, const w4<T>& C) {
  cx<T> j0 = R.c[0] * C.c[2] + R.c[1] * C.c[3] + R.c[2] * C.c[0] + R.c[3] * C.c[1];
  cx<T> j1 = R.c[0] * C.c[3] + R.c[1] * C.c[2] - R.c[2] * C.c[1] - R.c[3] * C.c[0];
  cx<T> j2 = mul_i(R.c[1] * C.c[2] + R.c[2] * C.c[1] - R.c[0] * C.c[3] - R.c[3] * C.c[0]);
  cx<T> j3 = R.c[0] * C.c[2] - R.c[1] * C.c[3] - R.c[2] * C.c[0] + R.c[3] * C.c[1];
  return w4<T>{{j0, j1, j2, j3}};
}
// vector current from a fermion pair: R gamma^nu C / P^2
template <class T> NLO_HD w4<T> ffv_vec(const w4<T>& R, const w4<T>& C, T den) {
  return den * ffv_cur(R, C);
}
// FFV amplitude R Vslash C
template <class T> NLO_HD cx<T> ffv_amp(const w4<T>& R, const w4<T>& V, const w4<T>& C) {
  return rdot(row_slash(R, V), C);
}
// three-vector current, legs (A, QA), (B, QB), off-shell leg with -(QA+QB):
// [(A.B)(QA-QB) + B (A.(QA+2QB)) - A (B.(2QA+QB))] / P^2
template <class T> NLO_HD w4<T> vvv_vec(const w4<T>& A, const r4<T>& QA, const w4<T>& B, const r4<T>& QB, T den) {
  r4<T> d1, d2, d3;
  for (int m = 0; m < 4; ++m) {
    d1.v[m] = QA.v[m] - QB.v[m];
    d2.v[m] = QA.v[m] + T(2) * QB.v[m];
    d3.v[m] = T(2) * QA.v[m] + QB.v[m];
  }
  cx<T> ab = mdot(A, B), a2 = mdot(A, d2), b3 = mdot(B, d3);
  w4<T> r;
  for (int m = 0; m < 4; ++m) r.c[m] = d1.v[m] * ab + B.c[m] * a2 - A.c[m] * b3;
  return den * r;
}
// three-vector amplitude V_{mu nu rho}(QA, QB, QL) A^mu B^nu L^rho
template <class T> NLO_HD cx<T> vvv_amp(const w4<T>& A, const r4<T>& QA, const w4<T>& B, const r4<T>& QB,
                                        const w4<T>& L, const r4<T>& QL) {
  r4<T> kp, pq, qk;
  for (int m = 0; m < 4; ++m) {
    kp.v[m] = QA.v[m] - QB.v[m];
    pq.v[m] = QB.v[m] - QL.v[m];
    qk.v[m] = QL.v[m] - QA.v[m];
  }
  return mdot(A, B) * mdot(L, kp) + mdot(B, L) * mdot(A, pq) + mdot(L, A) * mdot(B, qk);
}
// four-vector currents, legs A(mu), B(nu), C(rho), off-shell (sigma):
// structure 0 pairs (A,B)(C,.), 1 pairs (A,C)(B,.), 2 pairs (A,.)(B,C)
template <class T> NLO_HD w4<T> vvvv_vec0(const w4<T>& A, const w4<T>& B, const w4<T>& C, T den) {
  cx<T> ac = mdot(A, C), bc = mdot(B, C);
  return den * (ac * B - bc * A);
}
template <class T> NLO_HD w4<T> vvvv_vec1(const w4<T>& A, const w4<T>& B, const w4<T>& C, T den) {
  cx<T> ab = mdot(A, B), bc = mdot(B, C);
  return den * (ab * C - bc * A);
}
template <class T> NLO_HD w4<T> vvvv_vec2(const w4<T>& A, const w4<T>& B, const w4<T>& C, T den) {
  cx<T> ab = mdot(A, B), ac = mdot(A, C);
  return den * (ab * C - ac * B);
}
template <class T> NLO_HD cx<T> vvvv_amp0(const w4<T>& A, const w4<T>& B, const w4<T>& C, const w4<T>& L) {
  return mdot(A, C) * mdot(B, L) - mdot(B, C) * mdot(A, L);
}
template <class T> NLO_HD cx<T> vvvv_amp1(const w4<T>& A, const w4<T>& B, const w4<T>& C, const w4<T>& L) {
  return mdot(A, B) * mdot(C, L) - mdot(B, C) * mdot(A, L);
}
template <class T> NLO_HD cx<T> vvvv_amp2(const w4<T>& A, const w4<T>& B, const w4<T>& C, const w4<T>& L) {
  return mdot(A, B) * mdot(C, L) - mdot(A, C) * mdot(B, L);
}

// ---------------------------------------------------------------------------
// helicity-independent per-leg data, computed in FP64
// ---------------------------------------------------------------------------
NLO_HD void ferm_setup(const double* p, double m, ferm_data<double>& d) {
  double px = p[1], py = p[2], pz = p[3];
  double pt2 = px * px + py * py;
  double pa = sqrt(pt2 + pz * pz);
  double pp = (pz >= 0.0) ? pa + pz : pt2 / (pa - pz);   // |p| + pz without cancellation
  if (pp > 0.0) {
    double n = 1.0 / sqrt(2.0 * pa * pp);
    d.a = pp * n; d.br = px * n; d.bi = py * n;
  } else {                                             // p along -z
    d.a = 0.0; d.br = 1.0; d.bi = 0.0;
  }
  d.wp = sqrt(p[0] + pa);
  d.wm = (m == 0.0) ? 0.0 : m / d.wp;
}
NLO_HD void vec_setup(const double* p, vec_data<double>& d) {
  double px = p[1], py = p[2], pz = p[3];
  double pt = sqrt(px * px + py * py);
  double pa = sqrt(pt * pt + pz * pz);
  double ct = pz / pa, st = pt / pa;
  double cp = pt > 0.0 ? px / pt : 1.0, sp = pt > 0.0 ? py / pt : 0.0;
  const double s2 = 0.70710678118654752440;
  d.e1x = ct * cp * s2; d.e1y = ct * sp * s2; d.e1z = -st * s2;
  d.e2x = -sp * s2; d.e2y = cp * s2;
}
// multiply the wavefunction a leg's data builds by c
template <class T> NLO_HD void scale_leg(ferm_data<T>& d, T c) { d.wp = d.wp * c; d.wm = d.wm * c; }
template <class T> NLO_HD void scale_leg(vec_data<T>& d, T c) {
  d.e1x = d.e1x * c; d.e1y = d.e1y * c; d.e1z = d.e1z * c; d.e2x = d.e2x * c; d.e2y = d.e2y * c;
}
template <class T> NLO_HD ferm_data<T> cast(const ferm_data<double>& d) {
  return {T(d.a), T(d.br), T(d.bi), T(d.wp), T(d.wm)};
}
template <class T> NLO_HD vec_data<T> cast(const vec_data<double>& d) {
  return {T(d.e1x), T(d.e1y), T(d.e1z), T(d.e2x), T(d.e2y)};
}

}  // namespace nlo
