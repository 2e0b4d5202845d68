// CPU ORACLE for tree-level squared matrix elements -- TEST INFRASTRUCTURE.
//
// Only the tests, the smoke check and the benchmark's CPU-baseline leg may
// load this library.  It shares no code with the GPU path.  It is built twice
// from this file: in IEEE double, and (-DORACLE_QUAD) in IEEE binary128, the
// reference for the subtracted weight near the soft and collinear limits.
//
// What it computes (the paper's Born and real-emission equations: a tree
// amplitude is the sum of Feynman diagrams and the cross section follows
// from its absolute square):
//     |M|^2 = avg * sum_{helicities} sum_{colours} |sum_{diagrams} M|^2
// It sums every helicity combination (no filtering) and every colour.
//
// Two independent evaluations are provided:
//  * me2:        colour-ordered Berends-Giele recursion for one quark line plus
//                n gluons (gg->tt~, gg->tt~g, gg->tt~gg), contracted with a
//                colour matrix summed by brute force over explicit SU(3)
//                generators; explicit Feynman diagrams with explicit colour
//                tensors for the lepton and two-quark-line processes.
//  * me2_brute:  the full colour-dressed Feynman-rule recursion (f^{abc},
//                T^a, every external colour assignment summed explicitly),
//                i.e. the plain definition; slow, used to pin me2 on a few
//                events.
// Also: the FKS-subtracted real emission (fks, with colour-linked and
// spin-correlated Borns) and the RAMBO phase-space generator (rambo), each
// written out step by step further below.
//
// Conventions: metric (+,-,-,-); chiral Dirac representation; Feynman gauge;
// Peskin-Schroeder vertex rules: quark-gluon  i g gamma^mu T^a,
// fermion-photon  -i e Q gamma^mu, three-gluon
// g f^{abc}[g^{mu nu}(k-p)^rho + g^{nu rho}(p-q)^mu + g^{rho mu}(q-k)^nu]
// (momenta incoming), four-gluon -i g^2 [f^{abe}f^{cde}(...) + ...],
// propagators i(pslash+m)/(p^2-m^2) and -i g_{mu nu}/p^2.  T^a = lambda^a/2.
// External particles are on shell: a propagator denominator p^2 - m^2 is
// formed from the pairwise invariants 2 q_a.q_b and the nominal masses of the
// legs on one side of the line (den_of).
// Gamma_top = 0.  Helicity index h: bit (npart-1-k) of h set <=> leg k has
// helicity +1.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <functional>
#include <mutex>
#include <map>
#include <thread>
#include <vector>
#include <array>
#include <algorithm>

// ----------------------------------------------------------------------------
// scalar type
// ----------------------------------------------------------------------------
// The default build computes in IEEE double.  Built with -DORACLE_QUAD it
// computes in IEEE binary128 (__float128, libquadmath).  Near the soft and
// collinear limits the subtracted real emission is a difference of terms
// that each grow like 1/(xi (1-y)), so the weight keeps about
// log10(1/(xi (1-y))) fewer digits than the arithmetic carries; the paper
// names quadruple precision as the remedy for such losses in higher-order
// evaluations, and the binary128 build is the reference for that weight.
// Inputs and outputs are double in both builds.
#ifdef ORACLE_QUAD
#include <quadmath.h>
typedef __float128 Real;
static inline Real Sqrt(Real x) { return sqrtq(x); }
static inline Real Sin(Real x) { return sinq(x); }
static inline Real Cos(Real x) { return cosq(x); }
static inline Real Fabs(Real x) { return fabsq(x); }
static inline Real Pow(Real x, Real y) { return powq(x, y); }
static inline Real Log(Real x) { return logq(x); }
static const Real PI = 4 * atanq(Real(1));
#else
typedef double Real;
static inline Real Sqrt(Real x) { return std::sqrt(x); }
static inline Real Sin(Real x) { return std::sin(x); }
static inline Real Cos(Real x) { return std::cos(x); }
static inline Real Fabs(Real x) { return std::fabs(x); }
static inline Real Pow(Real x, Real y) { return std::pow(x, y); }
static inline Real Log(Real x) { return std::log(x); }
static const Real PI = M_PI;
#endif

// complex numbers over Real: the plain schoolbook operations
struct cd {
  Real re, im;
  cd(Real r = 0, Real i = 0) : re(r), im(i) {}
  Real real() const { return re; }
  Real imag() const { return im; }
  cd& operator+=(const cd& b) { re += b.re; im += b.im; return *this; }
  cd& operator-=(const cd& b) { re -= b.re; im -= b.im; return *this; }
};
static inline cd operator+(const cd& a, const cd& b) { return cd(a.re + b.re, a.im + b.im); }
static inline cd operator-(const cd& a, const cd& b) { return cd(a.re - b.re, a.im - b.im); }
static inline cd operator-(const cd& a) { return cd(-a.re, -a.im); }
static inline cd operator*(const cd& a, const cd& b) { return cd(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re); }
static inline cd operator*(Real a, const cd& b) { return cd(a * b.re, a * b.im); }
static inline cd operator*(const cd& a, Real b) { return cd(a.re * b, a.im * b); }
static inline cd operator/(const cd& a, Real b) { return cd(a.re / b, a.im / b); }
static inline cd operator/(const cd& a, const cd& b) {
  const Real d = b.re * b.re + b.im * b.im;
  return cd((a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d);
}
static inline bool operator==(const cd& a, const cd& b) { return a.re == b.re && a.im == b.im; }
static inline bool operator!=(const cd& a, const cd& b) { return !(a == b); }
static inline cd conj(const cd& a) { return cd(a.re, -a.im); }
static inline Real norm(const cd& a) { return a.re * a.re + a.im * a.im; }
static const cd I(0.0, 1.0);

// ----------------------------------------------------------------------------
// parameters
// ----------------------------------------------------------------------------
static Real g_alpha = 1.0 / 132.507;
static Real g_alpha_s = 0.118;
static Real g_mt = 173.0;

static Real e_qed() { return Sqrt(4.0 * PI * g_alpha); }
static Real g_qcd() { return Sqrt(4.0 * PI * g_alpha_s); }

// ----------------------------------------------------------------------------
// Lorentz algebra
// ----------------------------------------------------------------------------
struct V4 { Real v[4]; };                    // real four-vector
typedef std::array<cd, 4> C4;                   // complex four-vector (upper index) or spinor
typedef std::array<std::array<cd, 4>, 4> M4;    // 4x4 complex matrix

static Real dot(const V4& a, const V4& b) {
  return a.v[0] * b.v[0] - a.v[1] * b.v[1] - a.v[2] * b.v[2] - a.v[3] * b.v[3];
}
static cd cdot(const C4& a, const C4& b) {      // Minkowski product, no conjugation
  return a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
}
static cd cdot(const C4& a, const V4& b) {
  return a[0] * b.v[0] - a[1] * b.v[1] - a[2] * b.v[2] - a[3] * b.v[3];
}
static V4 vadd(const V4& a, const V4& b) { V4 r; for (int i = 0; i < 4; ++i) r.v[i] = a.v[i] + b.v[i]; return r; }
static V4 vneg(const V4& a) { V4 r; for (int i = 0; i < 4; ++i) r.v[i] = -a.v[i]; return r; }
static C4 c4(const V4& a) { C4 r; for (int i = 0; i < 4; ++i) r[i] = a.v[i]; return r; }
static C4 c4zero() { C4 r; r.fill(0.0); return r; }
static C4 add(const C4& a, const C4& b) { C4 r; for (int i = 0; i < 4; ++i) r[i] = a[i] + b[i]; return r; }
static C4 scale(cd s, const C4& a) { C4 r; for (int i = 0; i < 4; ++i) r[i] = s * a[i]; return r; }

// gamma matrices, chiral representation: gamma^0 = [[0,1],[1,0]],
// gamma^k = [[0, sigma^k], [-sigma^k, 0]]
static M4 GAMMA[4];
static void init_gamma() {
  static bool done = false;
  if (done) return;
  const cd sig[4][2][2] = {
      {{1, 0}, {0, 1}},
      {{0, 1}, {1, 0}},
      {{0, -I}, {I, 0}},
      {{1, 0}, {0, -1}}};
  for (int mu = 0; mu < 4; ++mu) {
    for (auto& row : GAMMA[mu]) row.fill(0.0);
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        if (mu == 0) {
          GAMMA[0][a][2 + b] = sig[0][a][b];
          GAMMA[0][2 + a][b] = sig[0][a][b];
        } else {
          GAMMA[mu][a][2 + b] = sig[mu][a][b];
          GAMMA[mu][2 + a][b] = -sig[mu][a][b];
        }
      }
  }
  done = true;
}

// gamma^mu a_mu
static M4 slash(const C4& a) {
  M4 r;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j)
      r[i][j] = GAMMA[0][i][j] * a[0] - GAMMA[1][i][j] * a[1] - GAMMA[2][i][j] * a[2] - GAMMA[3][i][j] * a[3];
  return r;
}
static M4 mmul(const M4& a, const M4& b) {
  M4 r;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      cd s = 0;
      for (int k = 0; k < 4; ++k) s += a[i][k] * b[k][j];
      r[i][j] = s;
    }
  return r;
}
static C4 mv(const M4& m, const C4& c) {       // matrix * column spinor
  C4 r;
  for (int i = 0; i < 4; ++i) { cd s = 0; for (int k = 0; k < 4; ++k) s += m[i][k] * c[k]; r[i] = s; }
  return r;
}
static C4 vm(const C4& row, const M4& m) {     // row spinor * matrix
  C4 r;
  for (int j = 0; j < 4; ++j) { cd s = 0; for (int k = 0; k < 4; ++k) s += row[k] * m[k][j]; r[j] = s; }
  return r;
}
static cd rc(const C4& row, const C4& col) { cd s = 0; for (int k = 0; k < 4; ++k) s += row[k] * col[k]; return s; }
// row gamma^mu col, for mu = 0..3 (upper index)
static C4 current(const C4& row, const C4& col) {
  C4 r;
  for (int mu = 0; mu < 4; ++mu) r[mu] = rc(row, mv(GAMMA[mu], col));
  return r;
}
// fermion propagator i(pslash + m)/(p^2 - m^2), p along the fermion-number
// arrow; d = p^2 - m^2 from the pairwise invariants (den_of below)
static M4 fprop(const V4& p, Real m, Real d) {
  M4 r = slash(c4(p));
  cd den = I / d;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) r[i][j] = (r[i][j] + (i == j ? cd(m) : cd(0))) * den;
  return r;
}

// ----------------------------------------------------------------------------
// external wavefunctions
// ----------------------------------------------------------------------------
// two-component helicity eigenstates of sigma.phat
static void chi(const V4& p, int lam, cd out[2]) {
  Real px = p.v[1], py = p.v[2], pz = p.v[3];
  Real pa = Sqrt(px * px + py * py + pz * pz);
  Real pt2 = px * px + py * py;
  Real pp = (pz >= 0) ? pa + pz : pt2 / (pa - pz);   // |p| + pz without cancellation
  if (pp <= 0.0) {                                      // p along -z
    if (lam > 0) { out[0] = 0; out[1] = 1; }
    else { out[0] = -1; out[1] = 0; }
    return;
  }
  Real nrm = 1.0 / Sqrt(2.0 * pa * pp);
  if (lam > 0) { out[0] = pp * nrm; out[1] = cd(px, py) * nrm; }
  else { out[0] = cd(-px, py) * nrm; out[1] = pp * nrm; }
}
static void omegas(const V4& p, Real m, Real& wp, Real& wm) {
  Real pa = Sqrt(p.v[1] * p.v[1] + p.v[2] * p.v[2] + p.v[3] * p.v[3]);
  wp = Sqrt(p.v[0] + pa);                     // sqrt(E + |p|)
  wm = (m == 0.0) ? 0.0 : m / wp;                  // sqrt(E - |p|), exact zero if massless
}
// u(p, lam): (sqrt(E - lam|p|) chi_lam, sqrt(E + lam|p|) chi_lam)
static C4 u_spinor(const V4& p, Real m, int lam) {
  Real wp, wm; omegas(p, m, wp, wm);
  cd x[2]; chi(p, lam, x);
  Real lo = lam > 0 ? wm : wp, hi = lam > 0 ? wp : wm;
  return C4{lo * x[0], lo * x[1], hi * x[0], hi * x[1]};
}
// v(p, lam): (-lam sqrt(E + lam|p|) chi_{-lam}, lam sqrt(E - lam|p|) chi_{-lam})
static C4 v_spinor(const V4& p, Real m, int lam) {
  Real wp, wm; omegas(p, m, wp, wm);
  cd x[2]; chi(p, -lam, x);
  Real a = lam > 0 ? wp : wm, b = lam > 0 ? wm : wp;
  Real l = lam;
  return C4{-l * a * x[0], -l * a * x[1], l * b * x[0], l * b * x[1]};
}
static C4 bar(const C4& s) {                      // s^dagger gamma^0
  C4 r;
  for (int j = 0; j < 4; ++j) { cd t = 0; for (int k = 0; k < 4; ++k) t += conj(s[k]) * GAMMA[0][k][j]; r[j] = t; }
  return r;
}
// massless vector polarisation eps(k, lam) = (-lam eps1 - i eps2)/sqrt2
static C4 polvec(const V4& k, int lam) {
  Real px = k.v[1], py = k.v[2], pz = k.v[3];
  Real pa = Sqrt(px * px + py * py + pz * pz);
  Real pt = Sqrt(px * px + py * py);
  Real ct = pz / pa, st = pt / pa;
  Real cp = pt > 0 ? px / pt : 1.0, sp = pt > 0 ? py / pt : 0.0;
  Real e1[4] = {0, ct * cp, ct * sp, -st};
  Real e2[4] = {0, -sp, cp, 0};
  C4 r;
  const Real s2 = 1.0 / Sqrt(2.0);
  for (int mu = 0; mu < 4; ++mu) r[mu] = (-Real(lam) * e1[mu] - I * e2[mu]) * s2;
  return r;
}
static C4 conjv(const C4& a) { C4 r; for (int i = 0; i < 4; ++i) r[i] = conj(a[i]); return r; }

// ----------------------------------------------------------------------------
// SU(3)
// ----------------------------------------------------------------------------
typedef std::array<std::array<cd, 3>, 3> M3;
static M3 TA[8];
static Real FABC[8][8][8];
static void init_su3() {
  static bool done = false;
  if (done) return;
  for (auto& t : TA) for (auto& r : t) r.fill(0.0);
  // Gell-Mann matrices / 2
  TA[0][0][1] = 0.5; TA[0][1][0] = 0.5;
  TA[1][0][1] = -0.5 * I; TA[1][1][0] = 0.5 * I;
  TA[2][0][0] = 0.5; TA[2][1][1] = -0.5;
  TA[3][0][2] = 0.5; TA[3][2][0] = 0.5;
  TA[4][0][2] = -0.5 * I; TA[4][2][0] = 0.5 * I;
  TA[5][1][2] = 0.5; TA[5][2][1] = 0.5;
  TA[6][1][2] = -0.5 * I; TA[6][2][1] = 0.5 * I;
  const Real r3 = 1.0 / Sqrt(3.0);
  TA[7][0][0] = 0.5 * r3; TA[7][1][1] = 0.5 * r3; TA[7][2][2] = -r3;
  // f^{abc} = -2 i Tr([T^a, T^b] T^c)
  for (int a = 0; a < 8; ++a)
    for (int b = 0; b < 8; ++b)
      for (int c = 0; c < 8; ++c) {
        cd tr = 0;
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k)
              tr += (TA[a][i][j] * TA[b][j][k] - TA[b][i][j] * TA[a][j][k]) * TA[c][k][i];
        Real f = (-2.0 * I * tr).real();
        FABC[a][b][c] = Fabs(f) < 1e-14 ? 0.0 : f;
      }
  done = true;
}

// ----------------------------------------------------------------------------
// process table
// ----------------------------------------------------------------------------
enum { EE_MUMU = 0, EE_UU, EE_UUG, GG_TT, UU_TT, GG_TTG, UU_TTG, UG_TTU, GG_TTGG, NPROC };

struct ProcDef {
  const char* name;
  int npart;
  int ncolour;          // dimension of the amplitude vector returned by flows()
  Real avg;           // initial spin x colour average
  Real ident;         // identical final-state particle factor (exported, not applied)
  int nin;
  // per leg: 'g' gluon, 'q' quark (fermion), 'Q' antiquark, 'l' lepton, 'L' antilepton
  const char* kinds;
  int a_pow, as_pow;    // |M|^2 scales as alpha^a alpha_s^b
};
static const ProcDef PROCS[NPROC] = {
    {"ee_mumu", 4, 1, 0.25, 1.0, 2, "lLlL", 2, 0},
    {"ee_uu", 4, 1, 0.25, 1.0, 2, "lLqQ", 2, 0},
    {"ee_uug", 5, 2, 0.25, 1.0, 2, "lLqQg", 2, 1},
    {"gg_tt", 4, 2, 1 / Real(256), 1.0, 2, "ggqQ", 0, 2},
    {"uu_tt", 4, 1, 1 / Real(36), 1.0, 2, "qQqQ", 0, 2},
    {"gg_ttg", 5, 6, 1 / Real(256), 1.0, 2, "ggqQg", 0, 3},
    {"uu_ttg", 5, 5, 1 / Real(36), 1.0, 2, "qQqQg", 0, 3},
    {"ug_ttu", 5, 5, 1 / Real(96), 1.0, 2, "qgqQq", 0, 3},
    {"gg_ttgg", 6, 24, 1 / Real(256), 0.5, 2, "ggqQgg", 0, 4},
};

static Real leg_mass(int proc, int k) {
  // tops are legs 2,3 of every gg/uu/ug process; everything else massless
  if (proc >= GG_TT && (k == 2 || k == 3)) return g_mt;
  return 0.0;
}

// Wavefunction of external leg k.  incoming momenta q_k = +p_k (initial),
// -p_k (final).  Fermion legs give the row or column spinor according to the
// particle and its direction; vector legs give eps (incoming) or eps* (outgoing).
struct Ext {
  V4 q[8];        // incoming momenta
  V4 p[8];        // physical momenta
  C4 w[8];        // wavefunction (vector: upper-index components; spinor: row or column)
  int n;          // number of legs
  Real m2[8];     // nominal squared mass of each leg
  Real s2[8][8];  // 2 q_a.q_b
};

// Denominator P^2 - m^2 of an internal line whose incoming momentum is the sum
// of the legs in `mask`.  External particles are on shell by definition, so
// P^2 = sum_a m_a^2 + sum_{a<b} 2 q_a.q_b over the legs of the line; by
// momentum conservation the complementary set gives the same value, and the
// smaller set is used (ties: the set holding leg 0).  The near-singular
// invariants of a soft or collinear emission (2 k_i.k_j, 2 k_i.p_l) are then
// differences of single pairwise products, never of O(s) squares, and the
// rounding of the input mass shells does not enter.
static Real den_of(const Ext& ex, unsigned mask, Real m) {
  const unsigned full = (1u << ex.n) - 1u;
  const unsigned comp = full & ~mask;
  const int a = __builtin_popcount(mask), b = __builtin_popcount(comp);
  if (b < a || (b == a && (comp & 1u))) mask = comp;
  Real d = -m * m;
  for (int x = 0; x < ex.n; ++x)
    if (mask >> x & 1u) d += ex.m2[x];
  for (int x = 0; x < ex.n; ++x)
    if (mask >> x & 1u)
      for (int y = x + 1; y < ex.n; ++y)
        if (mask >> y & 1u) d += ex.s2[x][y];
  return d;
}

// ----------------------------------------------------------------------------
// colour-ordered Berends-Giele recursion: one quark line + n gluons
// ----------------------------------------------------------------------------
// Colour decomposition M = sum_sigma (T^{a_sigma1} ... T^{a_sigman})_{i j} A(sigma),
// i the colour of the row end, j of the column end.  Colour-ordered rules
// (T normalised to Tr = 1/2) follow from the vertex rules above after
// f^{abc} = -2i Tr([T^a,T^b]T^c) and T^c_{ij}T^c_{kl} -> (1/2) d_il d_kj
// (the U(1) pieces cancel at tree level): quark vertex i g gamma^mu,
// ordered 3-gluon vertex -2 i g V_{mu nu rho}, ordered 4-gluon vertex
// 2 i g^2 (2 g^{mu rho} g^{nu sigma} - g^{mu sigma} g^{nu rho} - g^{mu nu} g^{rho sigma}),
// and a factor 1/2 per internal gluon line.
struct BGLine {
  int row, col;                   // leg indices of the row and column ends
  std::vector<int> gl;            // gluon leg indices
  Real m;                       // quark mass
};

static BGLine bg_line(int proc) {
  BGLine L;
  L.row = 2; L.col = 3; L.m = g_mt;
  if (proc == GG_TT) L.gl = {0, 1};
  else if (proc == GG_TTG) L.gl = {0, 1, 4};
  else L.gl = {0, 1, 4, 5};
  return L;
}

struct BGCache {
  int n;
  std::vector<char> have;
  std::vector<C4> J;
  std::vector<V4> Q;
  int key(const int* t, int len) const {
    int k = 0;
    for (int i = 0; i < len; ++i) k = k * (n + 1) + (t[i] + 1);
    return k;
  }
};

static C4 bg_current(BGCache& c, const Ext& ex, const BGLine& L, const int* t, int len, V4& Qout) {
  int k = c.key(t, len);
  if (c.have[k]) { Qout = c.Q[k]; return c.J[k]; }
  C4 J = c4zero();
  V4 Q{{0, 0, 0, 0}};
  unsigned mask = 0;
  for (int i = 0; i < len; ++i) { Q = vadd(Q, ex.q[L.gl[t[i]]]); mask |= 1u << L.gl[t[i]]; }
  if (len == 1) {
    J = ex.w[L.gl[t[0]]];
  } else {
    const Real g = g_qcd();
    Real P2 = den_of(ex, mask, 0.0);
    for (int s = 1; s < len; ++s) {           // three-gluon vertex, order (A, B, offshell)
      V4 QA, QB;
      C4 JA = bg_current(c, ex, L, t, s, QA);
      C4 JB = bg_current(c, ex, L, t + s, len - s, QB);
      cd ab = cdot(JA, JB);
      V4 d1, d2, d3;
      for (int m = 0; m < 4; ++m) {
        d1.v[m] = QA.v[m] - QB.v[m];
        d2.v[m] = QA.v[m] + 2.0 * QB.v[m];
        d3.v[m] = 2.0 * QA.v[m] + QB.v[m];
      }
      cd a2 = cdot(JA, d2), b3 = cdot(JB, d3);
      C4 V;
      for (int m = 0; m < 4; ++m) V[m] = ab * d1.v[m] + JB[m] * a2 - JA[m] * b3;
      // (-i/P^2)(1/2)(-2 i g) V = -g V / P^2
      J = add(J, scale(-g / P2, V));
    }
    for (int s1 = 1; s1 < len; ++s1)           // four-gluon vertex, order (A, B, C, offshell)
      for (int s2 = s1 + 1; s2 < len; ++s2) {
        V4 QA, QB, QC;
        C4 JA = bg_current(c, ex, L, t, s1, QA);
        C4 JB = bg_current(c, ex, L, t + s1, s2 - s1, QB);
        C4 JC = bg_current(c, ex, L, t + s2, len - s2, QC);
        cd ac = cdot(JA, JC), bc = cdot(JB, JC), ab = cdot(JA, JB);
        C4 V;
        for (int m = 0; m < 4; ++m) V[m] = 2.0 * ac * JB[m] - bc * JA[m] - ab * JC[m];
        // (-i/P^2)(1/2)(2 i g^2) V = g^2 V / P^2
        J = add(J, scale(g * g / P2, V));
      }
  }
  c.have[k] = 1; c.J[k] = J; c.Q[k] = Q;
  Qout = Q;
  return J;
}

// Row current after absorbing the ordered gluons t[0..len): R(A) = sum R(A') (i g Jslash(A'')) S(-Q)
static C4 bg_row(BGCache& c, std::map<int, C4>& rmemo, const Ext& ex, const BGLine& L, const int* t, int len) {
  if (len == 0) return ex.w[L.row];
  int k = c.key(t, len);
  auto it = rmemo.find(k);
  if (it != rmemo.end()) return it->second;
  const Real g = g_qcd();
  C4 acc = c4zero();
  for (int s = 0; s < len; ++s) {
    C4 R = bg_row(c, rmemo, ex, L, t, s);
    V4 Qd;
    C4 Jd = bg_current(c, ex, L, t + s, len - s, Qd);
    acc = add(acc, vm(R, slash(scale(I * g, Jd))));
  }
  V4 Q = ex.q[L.row];
  unsigned mask = 1u << L.row;
  for (int i = 0; i < len; ++i) { Q = vadd(Q, ex.q[L.gl[t[i]]]); mask |= 1u << L.gl[t[i]]; }
  C4 r = vm(acc, fprop(vneg(Q), L.m, den_of(ex, mask, L.m)));
  rmemo[k] = r;
  return r;
}

static void bg_flows(const BGLine& L, const Ext& ex, cd* out) {
  int n = (int)L.gl.size();
  BGCache c;
  c.n = n;
  int sz = 1;
  for (int i = 0; i < n; ++i) sz *= (n + 1);
  c.have.assign(sz, 0);
  c.J.resize(sz);
  c.Q.resize(sz);
  std::map<int, C4> rmemo;
  std::vector<int> perm(n);
  for (int i = 0; i < n; ++i) perm[i] = i;
  const Real g = g_qcd();
  int idx = 0;
  do {
    cd A = 0;
    for (int s = 0; s < n; ++s) {
      C4 R = bg_row(c, rmemo, ex, L, perm.data(), s);
      V4 Qd;
      C4 Jd = bg_current(c, ex, L, perm.data() + s, n - s, Qd);
      A += rc(vm(R, slash(scale(I * g, Jd))), ex.w[L.col]);
    }
    out[idx++] = A;
  } while (std::next_permutation(perm.begin(), perm.end()));
}

// colour matrix of the string basis, by brute force over explicit generators
static std::vector<Real> bg_colour_matrix(int n) {
  init_su3();
  std::vector<std::vector<int>> perms;
  std::vector<int> perm(n);
  for (int i = 0; i < n; ++i) perm[i] = i;
  do perms.push_back(perm); while (std::next_permutation(perm.begin(), perm.end()));
  int nc = (int)perms.size();
  std::vector<Real> C(nc * nc, 0.0);
  int nadj = 1;
  for (int i = 0; i < n; ++i) nadj *= 8;
  std::vector<M3> S(nc);
  std::vector<int> a(n);
  for (int code = 0; code < nadj; ++code) {
    int x = code;
    for (int i = 0; i < n; ++i) { a[i] = x % 8; x /= 8; }
    for (int p = 0; p < nc; ++p) {
      M3 m;
      for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) m[i][j] = (i == j) ? 1.0 : 0.0;
      for (int s = 0; s < n; ++s) {
        const M3& t = TA[a[perms[p][s]]];
        M3 r;
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j) { cd v = 0; for (int k = 0; k < 3; ++k) v += m[i][k] * t[k][j]; r[i][j] = v; }
        m = r;
      }
      S[p] = m;
    }
    for (int p = 0; p < nc; ++p)
      for (int q = 0; q < nc; ++q) {
        cd v = 0;
        for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) v += conj(S[p][i][j]) * S[q][i][j];
        C[p * nc + q] += v.real();
      }
  }
  return C;
}

// ----------------------------------------------------------------------------
// explicit diagrams with explicit colour tensors
// ----------------------------------------------------------------------------
// Two quark lines (light line 1 = (r1, c1), top line 2 = (r2, c2)) exchanging a
// gluon, with an optional extra gluon leg.  Returns the 5 diagram amplitudes
// (or 1 without the gluon); colour tensors are built by colour_tensors_2line.
struct TwoLine { int r1, c1, r2, c2, g; };

static TwoLine two_line(int proc) {
  if (proc == UU_TT) return TwoLine{1, 0, 2, 3, -1};
  if (proc == UU_TTG) return TwoLine{1, 0, 2, 3, 4};
  return TwoLine{4, 0, 2, 3, 1};                  // ug -> tt~u: row = outgoing u, col = incoming u
}

static void two_line_amps(int proc, const Ext& ex, cd* out) {
  TwoLine T = two_line(proc);
  const Real g = g_qcd();
  const Real m1 = 0.0, m2 = g_mt;
  const C4 &r1 = ex.w[T.r1], &c1 = ex.w[T.c1], &r2 = ex.w[T.r2], &c2 = ex.w[T.c2];
  V4 P1 = vadd(ex.q[T.r1], ex.q[T.c1]);
  V4 P2 = vadd(ex.q[T.r2], ex.q[T.c2]);
  const Real D1 = den_of(ex, (1u << T.r1) | (1u << T.c1), 0.0);
  const Real D2 = den_of(ex, (1u << T.r2) | (1u << T.c2), 0.0);
  if (T.g < 0) {
    // [r2 (i g gamma^mu) c2] (-i g_{mu nu}/P^2) [r1 (i g gamma^nu) c1]
    cd a = cdot(current(r2, c2), current(r1, c1)) * (I * g) * (I * g) * (-I / D1);
    out[0] = a;
    return;
  }
  const C4& eg = ex.w[T.g];
  const V4& qg = ex.q[T.g];
  M4 ge = slash(scale(I * g, eg));
  // D1: gluon on line 1, row side
  {
    C4 row = vm(vm(r1, ge), fprop(vneg(vadd(ex.q[T.r1], qg)), m1, den_of(ex, (1u << T.r1) | (1u << T.g), m1)));
    cd a = cdot(current(row, c1), current(r2, c2)) * (I * g) * (I * g) * (-I / D2);
    out[0] = a;
  }
  // D2: gluon on line 1, column side
  {
    C4 col = mv(fprop(vadd(ex.q[T.c1], qg), m1, den_of(ex, (1u << T.c1) | (1u << T.g), m1)), mv(ge, c1));
    cd a = cdot(current(r1, col), current(r2, c2)) * (I * g) * (I * g) * (-I / D2);
    out[1] = a;
  }
  // D3: gluon on line 2, row side
  {
    C4 row = vm(vm(r2, ge), fprop(vneg(vadd(ex.q[T.r2], qg)), m2, den_of(ex, (1u << T.r2) | (1u << T.g), m2)));
    cd a = cdot(current(row, c2), current(r1, c1)) * (I * g) * (I * g) * (-I / D1);
    out[2] = a;
  }
  // D4: gluon on line 2, column side
  {
    C4 col = mv(fprop(vadd(ex.q[T.c2], qg), m2, den_of(ex, (1u << T.c2) | (1u << T.g), m2)), mv(ge, c2));
    cd a = cdot(current(r2, col), current(r1, c1)) * (I * g) * (I * g) * (-I / D1);
    out[3] = a;
  }
  // D5: three-gluon vertex, legs (b, mu, P1), (c, nu, P2), (a, rho, qg)
  {
    C4 L1 = scale(I * g, current(r1, c1));
    C4 L2 = scale(I * g, current(r2, c2));
    // propagators -i/P^2 on the two exchanged gluons
    L1 = scale(-I / D1, L1);
    L2 = scale(-I / D2, L2);
    // V(k,p,q) contracted: (L1.L2)(k-p).eg + (L2.eg)(p-q).L1 + (eg.L1)(q-k).L2
    V4 kmp, pmq, qmk;
    for (int m = 0; m < 4; ++m) {
      kmp.v[m] = P1.v[m] - P2.v[m];
      pmq.v[m] = P2.v[m] - qg.v[m];
      qmk.v[m] = qg.v[m] - P1.v[m];
    }
    cd v = cdot(L1, L2) * cdot(eg, kmp) + cdot(L2, eg) * cdot(L1, pmq) + cdot(eg, L1) * cdot(L2, qmk);
    out[4] = g * v;
  }
}

// colour tensors c_D[i1][j1][i2][j2][a] for the two-line diagrams, and the
// colour matrix K_{DD'} = sum conj(c_D) c_D'
static std::vector<cd> two_line_colour_matrix(int proc) {
  init_su3();
  bool glu = (proc != UU_TT);
  int nd = glu ? 5 : 1;
  int na = glu ? 8 : 1;
  std::vector<cd> K(nd * nd, 0.0);
  for (int i1 = 0; i1 < 3; ++i1)
    for (int j1 = 0; j1 < 3; ++j1)
      for (int i2 = 0; i2 < 3; ++i2)
        for (int j2 = 0; j2 < 3; ++j2)
          for (int a = 0; a < na; ++a) {
            cd c[5] = {0, 0, 0, 0, 0};
            for (int b = 0; b < 8; ++b) {
              if (!glu) { c[0] += TA[b][i1][j1] * TA[b][i2][j2]; continue; }
              cd ab1 = 0, ba1 = 0, ab2 = 0, ba2 = 0;
              for (int k = 0; k < 3; ++k) {
                ab1 += TA[a][i1][k] * TA[b][k][j1];
                ba1 += TA[b][i1][k] * TA[a][k][j1];
                ab2 += TA[a][i2][k] * TA[b][k][j2];
                ba2 += TA[b][i2][k] * TA[a][k][j2];
              }
              c[0] += ab1 * TA[b][i2][j2];
              c[1] += ba1 * TA[b][i2][j2];
              c[2] += TA[b][i1][j1] * ab2;
              c[3] += TA[b][i1][j1] * ba2;
              for (int cc = 0; cc < 8; ++cc)
                if (FABC[b][cc][a] != 0.0) c[4] += TA[b][i1][j1] * TA[cc][i2][j2] * FABC[b][cc][a];
            }
            for (int d = 0; d < nd; ++d)
              for (int e = 0; e < nd; ++e) K[d * nd + e] += conj(c[d]) * c[e];
          }
  return K;
}

// e+e- -> f fbar (g) through one photon
static void ee_amps(int proc, const Ext& ex, cd* out) {
  const Real e = e_qed(), g = g_qcd();
  const Real Qe = -1.0;
  const Real Qf = (proc == EE_MUMU) ? Real(-1) : Real(2) / 3;
  // lepton current vbar(e+) gamma^nu u(e-): row = leg 1, column = leg 0
  C4 Lc = scale(-I * e * Qe, current(ex.w[1], ex.w[0]));
  V4 P = vadd(ex.q[0], ex.q[1]);
  C4 Lp = scale(-I / den_of(ex, 3u, 0.0), Lc);                 // photon propagator
  if (proc != EE_UUG) {
    out[0] = cdot(scale(-I * e * Qf, current(ex.w[2], ex.w[3])), Lp);
    return;
  }
  M4 ge = slash(scale(I * g, ex.w[4]));
  // D1: gluon on the outgoing quark (row, leg 2)
  C4 row = vm(vm(ex.w[2], ge), fprop(vneg(vadd(ex.q[2], ex.q[4])), 0.0, den_of(ex, (1u << 2) | (1u << 4), 0.0)));
  out[0] = cdot(scale(-I * e * Qf, current(row, ex.w[3])), Lp);
  // D2: gluon on the outgoing antiquark (column, leg 3)
  C4 col = mv(fprop(vadd(ex.q[3], ex.q[4]), 0.0, den_of(ex, (1u << 3) | (1u << 4), 0.0)), mv(ge, ex.w[3]));
  out[1] = cdot(scale(-I * e * Qf, current(ex.w[2], col)), Lp);
}

// ----------------------------------------------------------------------------
// generic per-event evaluation
// ----------------------------------------------------------------------------
static int helicity_of(int h, int npart, int k) { return ((h >> (npart - 1 - k)) & 1) ? +1 : -1; }

// Build external wavefunctions for helicity h.  override_leg >= 0 replaces that
// vector leg's polarisation by override_vec (gauge and spin-correlation tests).
static void build_ext(int proc, const V4* p, int h, Ext& ex, int override_leg, const C4* override_vec) {
  const ProcDef& P = PROCS[proc];
  ex.n = P.npart;
  for (int k = 0; k < P.npart; ++k) {
    const Real mk = leg_mass(proc, k);
    ex.m2[k] = mk * mk;
    ex.q[k] = k < P.nin ? p[k] : vneg(p[k]);
  }
  for (int a = 0; a < P.npart; ++a)
    for (int b = a + 1; b < P.npart; ++b) ex.s2[a][b] = 2.0 * dot(ex.q[a], ex.q[b]);
  for (int k = 0; k < P.npart; ++k) {
    bool in = k < P.nin;
    ex.p[k] = p[k];
    int lam = helicity_of(h, P.npart, k);
    Real m = leg_mass(proc, k);
    char kind = P.kinds[k];
    if (kind == 'g') {
      C4 e = polvec(p[k], lam);
      ex.w[k] = in ? e : conjv(e);
      if (k == override_leg) ex.w[k] = *override_vec;
    } else if (kind == 'q' || kind == 'l') {
      // particle: incoming -> column u(p); outgoing -> row ubar(p)
      ex.w[k] = in ? u_spinor(p[k], m, lam) : bar(u_spinor(p[k], m, lam));
    } else {
      // antiparticle: incoming -> row vbar(p); outgoing -> column v(p)
      ex.w[k] = in ? bar(v_spinor(p[k], m, lam)) : v_spinor(p[k], m, lam);
    }
  }
}

struct ColourData {
  int nc;
  std::vector<cd> C;     // nc x nc hermitian
};
static ColourData COLOUR[NPROC];
static void init_colour() {
  static bool done = false;
  if (done) return;
  init_gamma();
  init_su3();
  for (int p = 0; p < NPROC; ++p) {
    ColourData& cdat = COLOUR[p];
    cdat.nc = PROCS[p].ncolour;
    cdat.C.assign(cdat.nc * cdat.nc, 0.0);
    if (p == GG_TT || p == GG_TTG || p == GG_TTGG) {
      int n = (p == GG_TT) ? 2 : (p == GG_TTG ? 3 : 4);
      std::vector<Real> C = bg_colour_matrix(n);
      for (size_t i = 0; i < C.size(); ++i) cdat.C[i] = C[i];
    } else if (p == UU_TT || p == UU_TTG || p == UG_TTU) {
      cdat.C = two_line_colour_matrix(p);
    } else if (p == EE_UUG) {
      // both diagrams carry T^a_{ij}: sum |T^a_ij|^2 = Tr(T^a T^a) = 4
      for (auto& x : cdat.C) x = 4.0;
    } else if (p == EE_UU) {
      cdat.C[0] = 3.0;     // delta_ij delta_ij
    } else {
      cdat.C[0] = 1.0;
    }
  }
  done = true;
}

static void flows(int proc, const Ext& ex, cd* out) {
  switch (proc) {
    case EE_MUMU: case EE_UU: case EE_UUG: ee_amps(proc, ex, out); break;
    case UU_TT: case UU_TTG: case UG_TTU: two_line_amps(proc, ex, out); break;
    default: bg_flows(bg_line(proc), ex, out); break;
  }
}

static Real quad(const ColourData& c, const cd* A) {
  cd s = 0;
  for (int i = 0; i < c.nc; ++i)
    for (int j = 0; j < c.nc; ++j) s += conj(A[i]) * c.C[i * c.nc + j] * A[j];
  return s.real();
}

static void load_event(const double* mom, int64_t ld, int64_t e, int npart, V4* p) {
  for (int k = 0; k < npart; ++k)
    for (int mu = 0; mu < 4; ++mu) p[k].v[mu] = mom[(k * 4 + mu) * ld + e];
}

// sum over helicities of the colour-summed |M_h|^2, times the average factor
static Real me2_event(int proc, const V4* p, Real* per_hel) {
  const ProcDef& P = PROCS[proc];
  const ColourData& c = COLOUR[proc];
  int nh = 1 << P.npart;
  std::vector<cd> A(c.nc);
  Real sum = 0;
  Ext ex;
  for (int h = 0; h < nh; ++h) {
    build_ext(proc, p, h, ex, -1, nullptr);
    flows(proc, ex, A.data());
    Real v = quad(c, A.data());
    if (per_hel) per_hel[h] = v * P.avg;
    sum += v;
  }
  return sum * P.avg;
}

template <class F>
static void parallel_for(int64_t n, int nthreads, F f) {
  if (nthreads <= 1 || n < 2) { for (int64_t i = 0; i < n; ++i) f(i); return; }
  std::vector<std::thread> th;
  int64_t chunk = (n + nthreads - 1) / nthreads;
  for (int t = 0; t < nthreads; ++t) {
    int64_t lo = t * chunk, hi = std::min(n, lo + chunk);
    if (lo >= hi) break;
    th.emplace_back([=, &f]() { for (int64_t i = lo; i < hi; ++i) f(i); });
  }
  for (auto& x : th) x.join();
}

// ----------------------------------------------------------------------------
// colour-dressed brute force (full Feynman rules, explicit colours)
// ----------------------------------------------------------------------------
// Currents over subsets of gluons carry an explicit adjoint index; the quark
// row current carries a fundamental index.  Summing the recursion equals
// summing all Feynman diagrams; every external colour assignment is summed.
struct Brute {
  const BGLine* L;
  const Ext* ex;
  int n;
  int ag[4];                        // external gluon colours
  std::vector<std::array<C4, 8>> G; // gluon currents per subset mask
  std::vector<V4> GQ;
  std::vector<char> gh;
  std::vector<std::array<C4, 3>> R; // row currents per subset mask
  std::vector<char> rh;
};

static void brute_gluon(Brute& b, int mask) {
  if (b.gh[mask]) return;
  const Ext& ex = *b.ex;
  const BGLine& L = *b.L;
  std::array<C4, 8> J;
  for (auto& x : J) x = c4zero();
  V4 Q{{0, 0, 0, 0}};
  int cnt = 0, only = -1;
  unsigned legs = 0;
  for (int i = 0; i < b.n; ++i)
    if (mask >> i & 1) { Q = vadd(Q, ex.q[L.gl[i]]); ++cnt; only = i; legs |= 1u << L.gl[i]; }
  if (cnt == 1) {
    J[b.ag[only]] = ex.w[L.gl[only]];
  } else {
    const Real g = g_qcd();
    Real P2 = den_of(ex, legs, 0.0);
    // 3-vertex, unordered splits: s1 contains the lowest set bit
    int low = mask & -mask;
    for (int s1 = (mask - 1) & mask; s1 > 0; s1 = (s1 - 1) & mask) {
      if (!(s1 & low)) continue;
      int s2 = mask ^ s1;
      brute_gluon(b, s1); brute_gluon(b, s2);
      const V4 &Q1 = b.GQ[s1], &Q2 = b.GQ[s2];
      V4 Q3 = vneg(vadd(Q1, Q2));
      V4 kmp, pmq, qmk;
      for (int m = 0; m < 4; ++m) { kmp.v[m] = Q1.v[m] - Q2.v[m]; pmq.v[m] = Q2.v[m] - Q3.v[m]; qmk.v[m] = Q3.v[m] - Q1.v[m]; }
      for (int c1 = 0; c1 < 8; ++c1)
        for (int c2 = 0; c2 < 8; ++c2) {
          const C4 &A = b.G[s1][c1], &B = b.G[s2][c2];
          if (A[0] == 0.0 && A[1] == 0.0 && A[2] == 0.0 && A[3] == 0.0) continue;
          if (B[0] == 0.0 && B[1] == 0.0 && B[2] == 0.0 && B[3] == 0.0) continue;
          // V_rho = (A.B)(k-p)_rho + B_rho (p-q).A + A_rho (q-k).B
          cd ab = cdot(A, B), pa = cdot(A, pmq), qb = cdot(B, qmk);
          C4 V;
          for (int m = 0; m < 4; ++m) V[m] = ab * kmp.v[m] + B[m] * pa + A[m] * qb;
          for (int c = 0; c < 8; ++c) {
            Real f = FABC[c1][c2][c];
            if (f == 0.0) continue;
            J[c] = add(J[c], scale((-I / P2) * g * f, V));
          }
        }
    }
    // 4-vertex, unordered 3-partitions
    std::vector<int> bits;
    for (int i = 0; i < b.n; ++i) if (mask >> i & 1) bits.push_back(i);
    int nb = (int)bits.size();
    if (nb >= 3) {
      std::vector<int> lab(nb, 0);
      int total = 1;
      for (int i = 0; i < nb; ++i) total *= 3;
      for (int code = 0; code < total; ++code) {
        int x = code;
        int m3[3] = {0, 0, 0};
        for (int i = 0; i < nb; ++i) { m3[x % 3] |= 1 << bits[i]; x /= 3; }
        if (!m3[0] || !m3[1] || !m3[2]) continue;
        // canonical: lowest bits ordered m3[0] < m3[1] < m3[2]
        auto lowb = [](int m) { return m & -m; };
        if (!(lowb(m3[0]) < lowb(m3[1]) && lowb(m3[1]) < lowb(m3[2]))) continue;
        for (int s = 0; s < 3; ++s) brute_gluon(b, m3[s]);
        for (int c1 = 0; c1 < 8; ++c1)
          for (int c2 = 0; c2 < 8; ++c2)
            for (int c3 = 0; c3 < 8; ++c3) {
              const C4 &A = b.G[m3[0]][c1], &B = b.G[m3[1]][c2], &C = b.G[m3[2]][c3];
              cd ab = cdot(A, B), ac = cdot(A, C), bc = cdot(B, C);
              if (ab == 0.0 && ac == 0.0 && bc == 0.0) continue;
              for (int d = 0; d < 8; ++d) {
                // legs a=A(mu), b=B(nu), c=C(rho), d=offshell(sigma)
                Real f1 = 0, f2 = 0, f3 = 0;
                for (int e = 0; e < 8; ++e) {
                  f1 += FABC[c1][c2][e] * FABC[c3][d][e];
                  f2 += FABC[c1][c3][e] * FABC[c2][d][e];
                  f3 += FABC[c1][d][e] * FABC[c2][c3][e];
                }
                if (f1 == 0 && f2 == 0 && f3 == 0) continue;
                C4 V;
                for (int m = 0; m < 4; ++m)
                  V[m] = f1 * (ac * B[m] - A[m] * bc) + f2 * (ab * C[m] - A[m] * bc) + f3 * (ab * C[m] - ac * B[m]);
                // (-i/P^2)(-i g^2) V = -g^2 V / P^2
                J[d] = add(J[d], scale(-g * g / P2, V));
              }
            }
      }
    }
  }
  b.G[mask] = J;
  b.GQ[mask] = Q;
  b.gh[mask] = 1;
}

static void brute_row(Brute& b, int mask, int irow) {
  if (b.rh[mask]) return;
  const Ext& ex = *b.ex;
  const BGLine& L = *b.L;
  std::array<C4, 3> R;
  for (auto& x : R) x = c4zero();
  if (mask == 0) {
    R[irow] = ex.w[L.row];
  } else {
    const Real g = g_qcd();
    std::array<C4, 3> acc;
    for (auto& x : acc) x = c4zero();
    for (int sg = mask; sg > 0; sg = (sg - 1) & mask) {   // gluons absorbed at the last vertex
      int sr = mask ^ sg;
      brute_row(b, sr, irow);
      brute_gluon(b, sg);
      for (int c = 0; c < 8; ++c) {
        const C4& G = b.G[sg][c];
        if (G[0] == 0.0 && G[1] == 0.0 && G[2] == 0.0 && G[3] == 0.0) continue;
        M4 gs = slash(scale(I * g, G));
        for (int j = 0; j < 3; ++j) {
          C4 t = vm(b.R[sr][j], gs);
          for (int k = 0; k < 3; ++k)
            if (TA[c][j][k] != 0.0) acc[k] = add(acc[k], scale(TA[c][j][k], t));
        }
      }
    }
    V4 Q = ex.q[L.row];
    unsigned legs = 1u << L.row;
    for (int i = 0; i < b.n; ++i) if (mask >> i & 1) { Q = vadd(Q, ex.q[L.gl[i]]); legs |= 1u << L.gl[i]; }
    M4 S = fprop(vneg(Q), L.m, den_of(ex, legs, L.m));
    for (int k = 0; k < 3; ++k) R[k] = vm(acc[k], S);
  }
  b.R[mask] = R;
  b.rh[mask] = 1;
}

static Real brute_event_hel(int proc, const V4* p, int h) {
  BGLine L = bg_line(proc);
  Ext ex;
  build_ext(proc, p, h, ex, -1, nullptr);
  int n = (int)L.gl.size();
  int full = (1 << n) - 1;
  int ncol = 1;
  for (int i = 0; i < n; ++i) ncol *= 8;
  const Real g = g_qcd();
  Real sum = 0;
  for (int code = 0; code < ncol; ++code) {
    Brute b;
    b.L = &L; b.ex = &ex; b.n = n;
    int x = code;
    for (int i = 0; i < n; ++i) { b.ag[i] = x % 8; x /= 8; }
    b.G.assign(1 << n, std::array<C4, 8>{});
    b.GQ.assign(1 << n, V4{});
    b.gh.assign(1 << n, 0);
    for (int irow = 0; irow < 3; ++irow) {
      b.R.assign(1 << n, std::array<C4, 3>{});
      b.rh.assign(1 << n, 0);
      cd M[3] = {0, 0, 0};
      for (int sg = full; sg > 0; sg = (sg - 1) & full) {
        int sr = full ^ sg;
        brute_row(b, sr, irow);
        brute_gluon(b, sg);
        for (int c = 0; c < 8; ++c) {
          const C4& G = b.G[sg][c];
          if (G[0] == 0.0 && G[1] == 0.0 && G[2] == 0.0 && G[3] == 0.0) continue;
          M4 gs = slash(scale(I * g, G));
          for (int j = 0; j < 3; ++j) {
            cd t = rc(vm(b.R[sr][j], gs), ex.w[L.col]);
            for (int k = 0; k < 3; ++k) M[k] += TA[c][j][k] * t;
          }
        }
      }
      for (int k = 0; k < 3; ++k) sum += norm(M[k]);
    }
  }
  return sum;
}

// ----------------------------------------------------------------------------
// C ABI (test infrastructure)
// ----------------------------------------------------------------------------
extern "C" {

int orc_nproc() { return NPROC; }

const char* orc_proc_name(int proc) { return (proc >= 0 && proc < NPROC) ? PROCS[proc].name : nullptr; }

void orc_set_params(double alpha, double alpha_s, double m_top) {
  g_alpha = alpha; g_alpha_s = alpha_s; g_mt = m_top;
}

int orc_proc_info(int proc, int* npart, int* ncolour, double* avg, double* ident, int* a_pow, int* as_pow) {
  if (proc < 0 || proc >= NPROC) return 1;
  const ProcDef& P = PROCS[proc];
  *npart = P.npart; *ncolour = P.ncolour; *avg = P.avg; *ident = P.ident;
  *a_pow = P.a_pow; *as_pow = P.as_pow;
  return 0;
}

// mom: [npart][4][ld] SoA; out[n]
int orc_me2(int proc, int64_t n, int64_t ld, const double* mom, double* out, int nthreads) {
  if (proc < 0 || proc >= NPROC) return 1;
  init_colour();
  const int np = PROCS[proc].npart;
  parallel_for(n, nthreads, [&](int64_t e) {
    V4 p[8];
    load_event(mom, ld, e, np, p);
    out[e] = me2_event(proc, p, nullptr);
  });
  return 0;
}

// per-helicity colour-summed values times the average: out[h * n + e]
int orc_me2_hel(int proc, int64_t n, int64_t ld, const double* mom, double* out, int nthreads) {
  if (proc < 0 || proc >= NPROC) return 1;
  init_colour();
  const int np = PROCS[proc].npart;
  const int nh = 1 << np;
  parallel_for(n, nthreads, [&](int64_t e) {
    V4 p[8];
    load_event(mom, ld, e, np, p);
    std::vector<Real> ph(nh);
    me2_event(proc, p, ph.data());
    for (int h = 0; h < nh; ++h) out[h * n + e] = ph[h];
  });
  return 0;
}

// colour-flow (or diagram) amplitude vector for one event (AoS p[npart][4]) and
// helicity h; override_leg >= 0 replaces that vector leg's wavefunction by
// ovec (4 complex as 8 doubles, upper index).  out: 2*ncolour doubles.
int orc_flows(int proc, const double* p_aos, int h, int override_leg, const double* ovec, double* out) {
  if (proc < 0 || proc >= NPROC) return 1;
  init_colour();
  const ProcDef& P = PROCS[proc];
  V4 p[8];
  for (int k = 0; k < P.npart; ++k) for (int mu = 0; mu < 4; ++mu) p[k].v[mu] = p_aos[k * 4 + mu];
  C4 ov;
  if (override_leg >= 0) for (int mu = 0; mu < 4; ++mu) ov[mu] = cd(ovec[2 * mu], ovec[2 * mu + 1]);
  Ext ex;
  build_ext(proc, p, h, ex, override_leg, &ov);
  std::vector<cd> A(P.ncolour);
  flows(proc, ex, A.data());
  for (int i = 0; i < P.ncolour; ++i) { out[2 * i] = A[i].real(); out[2 * i + 1] = A[i].imag(); }
  return 0;
}

// colour matrix of the amplitude vector (2*nc*nc doubles: re, im)
int orc_colour_matrix(int proc, double* out) {
  if (proc < 0 || proc >= NPROC) return 1;
  init_colour();
  const ColourData& c = COLOUR[proc];
  for (int i = 0; i < c.nc * c.nc; ++i) { out[2 * i] = c.C[i].real(); out[2 * i + 1] = c.C[i].imag(); }
  return 0;
}

// external wavefunction of leg k at helicity lam (+-1) for an event (AoS):
// 8 doubles (4 complex).  Used by the wavefunction pins.
int orc_wavefunction(int proc, const double* p_aos, int k, int lam, double* out) {
  if (proc < 0 || proc >= NPROC) return 1;
  init_colour();
  const ProcDef& P = PROCS[proc];
  V4 p[8];
  for (int j = 0; j < P.npart; ++j) for (int mu = 0; mu < 4; ++mu) p[j].v[mu] = p_aos[j * 4 + mu];
  int h = 0;
  if (lam > 0) h |= 1 << (P.npart - 1 - k);
  Ext ex;
  build_ext(proc, p, h, ex, -1, nullptr);
  for (int mu = 0; mu < 4; ++mu) { out[2 * mu] = ex.w[k][mu].real(); out[2 * mu + 1] = ex.w[k][mu].imag(); }
  return 0;
}

// colour-dressed brute force: raw sum over colours for helicity h (h < 0: all
// helicities), times the average factor.  gg processes only.
int orc_me2_brute(int proc, int64_t n, int64_t ld, const double* mom, int h, double* out, int nthreads) {
  if (proc != GG_TT && proc != GG_TTG && proc != GG_TTGG) return 1;
  init_colour();
  const int np = PROCS[proc].npart;
  const int nh = 1 << np;
  parallel_for(n, nthreads, [&](int64_t e) {
    V4 p[8];
    load_event(mom, ld, e, np, p);
    Real s = 0;
    if (h >= 0) s = brute_event_hel(proc, p, h);
    else for (int hh = 0; hh < nh; ++hh) s += brute_event_hel(proc, p, hh);
    out[e] = s * PROCS[proc].avg;
  });
  return 0;
}

}  // extern "C"

// ============================================================================
// FKS subtraction (ORACLE) -- the paper names FKS subtraction as the scheme
// whose soft and collinear counterterms make the real emission locally
// integrable, and splits the phase space into FKS sectors.  The paper does
// not spell out maps, sector functions or plus-distribution parameters; the
// fixed reading implemented here:
//   xi = 2 k_i^0 / sqrt(s_R) in the real partonic frame, y = cos(k_i, k_j)
//   (final j) or cos(k_i, beam 1) (initial j), phi = azimuth of k_i about the
//   emitter direction measured from the (emitter, z) plane.
//   FSR map: recoil boost along the emitter direction; ISR map: s_R =
//   s_B/(1-xi), Born final state pure-boosted to K = p1 + p2 - k_i.
//   xi = xi_tilde * xi_max; xi_max = 1 - M_rec^2/s (FSR), 1 - s_B/s_cap with
//   sqrt(s_cap) = 4000 GeV (ISR).
//   f(xi, y) = xi^2 (1-y) |M_R|^2 S_ij (FSR), xi^2 (1-y^2) |M_R|^2 S_i0 (ISR);
//   always-subtract (xi_c = xi_max, delta = 2):
//   W_FSR = [f(xi,y) - f(0,y) - f(xi,1) + f(0,1)] / (xi (1-y))
//   W_ISR = [f(xi,y) - f(0,y) - (1+y)/2 (f(xi,1) - f(0,1))
//                              - (1-y)/2 (f(xi,-1) - f(0,-1))] / (xi (1-y^2))
//   Sector functions S_ij = (h_ij/d_ij) / sum_P (h_kl/d_kl), d_kl = xi_k xi_l
//   (1-y_kl) (final l), xi_k (1-y_k^2) (beams), h = xi_l/(xi_k+xi_l) for
//   gluon-gluon pairs, else 1.
// The soft limit uses the eikonal factor with colour-linked Borns, the
// collinear limits the Altarelli-Parisi kernels with the spin-correlated Born
// for gluon splittings.
// ============================================================================
static const Real FKS_SQRT_SCAP = 4000.0;

// colour charge operators on explicit colour tensors ---------------------------
// leg kinds: 'r' fundamental (row end), 'c' antifundamental (column end),
// 'g' adjoint.  T^a acts as T^a on 'r', as -(T^a)^T on 'c', as -i f^{abc} on 'g'.
struct ColTensor {
  std::vector<char> kind;    // per coloured leg
  std::vector<int> dim;
  std::vector<cd> v;         // row-major over legs
};
static size_t ct_size(const ColTensor& t) { size_t s = 1; for (int d : t.dim) s *= d; return s; }
static ColTensor apply_charge(const ColTensor& t, int leg, int a) {
  ColTensor r = t;
  std::fill(r.v.begin(), r.v.end(), cd(0));
  size_t n = ct_size(t);
  size_t stride = 1;
  for (int k = (int)t.dim.size() - 1; k > leg; --k) stride *= t.dim[k];
  int d = t.dim[leg];
  for (size_t idx = 0; idx < n; ++idx) {
    if (t.v[idx] == 0.0) continue;
    int c = (int)((idx / stride) % d);
    size_t base = idx - (size_t)c * stride;
    for (int c2 = 0; c2 < d; ++c2) {
      cd f;
      if (t.kind[leg] == 'r') f = TA[a][c2][c];             // (T^a X)_{c2} = T^a_{c2 c} X_c
      else if (t.kind[leg] == 'c') f = -TA[a][c][c2];       // -(X T^a)_{c2} = -X_c T^a_{c c2}
      else f = -I * FABC[a][c2][c];                          // (F^a)_{c2 c} = -i f^{a c2 c}
      if (f != 0.0) r.v[base + (size_t)c2 * stride] += f * t.v[idx];
    }
  }
  return r;
}
static cd ct_dot(const ColTensor& a, const ColTensor& b) {
  cd s = 0;
  for (size_t i = 0; i < a.v.size(); ++i) s += conj(a.v[i]) * b.v[i];
  return s;
}

// explicit colour tensors of the amplitude basis of a Born process, legs in
// process order (coloured legs only), and the process-leg index of each
struct BornColour {
  std::vector<int> legs;              // process leg index of each coloured leg
  std::vector<ColTensor> basis;
  std::vector<std::vector<cd>> Ckl;   // per pair (k,l) over coloured legs, nc x nc
};

static void build_basis(int proc, BornColour& bc) {
  init_su3();
  bc.basis.clear();
  if (proc == EE_UU) {
    bc.legs = {2, 3};
    ColTensor t; t.kind = {'r', 'c'}; t.dim = {3, 3}; t.v.assign(9, 0.0);
    for (int i = 0; i < 3; ++i) t.v[i * 3 + i] = 1.0;
    bc.basis.push_back(t);
  } else if (proc == GG_TT || proc == GG_TTG) {
    BGLine L = bg_line(proc);
    int n = (int)L.gl.size();
    // coloured legs in process order
    bc.legs.clear();
    for (int k = 0; k < PROCS[proc].npart; ++k) bc.legs.push_back(k);
    std::vector<int> perm(n);
    for (int i = 0; i < n; ++i) perm[i] = i;
    do {
      ColTensor t;
      for (int k : bc.legs) {
        if (k == L.row) { t.kind.push_back('r'); t.dim.push_back(3); }
        else if (k == L.col) { t.kind.push_back('c'); t.dim.push_back(3); }
        else { t.kind.push_back('g'); t.dim.push_back(8); }
      }
      t.v.assign(ct_size(t), 0.0);
      // position of each gluon leg in the tensor
      std::vector<int> gpos(n);
      for (int g = 0; g < n; ++g)
        for (size_t q = 0; q < bc.legs.size(); ++q) if (bc.legs[q] == L.gl[g]) gpos[g] = (int)q;
      int rpos = -1, cpos = -1;
      for (size_t q = 0; q < bc.legs.size(); ++q) { if (bc.legs[q] == L.row) rpos = (int)q; if (bc.legs[q] == L.col) cpos = (int)q; }
      size_t N = ct_size(t);
      std::vector<int> idx(t.dim.size());
      for (size_t lin = 0; lin < N; ++lin) {
        size_t x = lin;
        for (int q = (int)t.dim.size() - 1; q >= 0; --q) { idx[q] = (int)(x % t.dim[q]); x /= t.dim[q]; }
        M3 m;
        for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) m[i][j] = (i == j) ? 1.0 : 0.0;
        for (int s = 0; s < n; ++s) {
          const M3& T = TA[idx[gpos[perm[s]]]];
          M3 r;
          for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) { cd v = 0; for (int k = 0; k < 3; ++k) v += m[i][k] * T[k][j]; r[i][j] = v; }
          m = r;
        }
        t.v[lin] = m[idx[rpos]][idx[cpos]];
      }
      bc.basis.push_back(t);
    } while (std::next_permutation(perm.begin(), perm.end()));
  } else if (proc == UU_TT) {
    // single diagram, colour sum_b T^b_{i1 j1} T^b_{i2 j2}; legs 0 u(in, col), 1 ubar(in, row), 2 t(row), 3 tbar(col)
    bc.legs = {0, 1, 2, 3};
    ColTensor t; t.kind = {'c', 'r', 'r', 'c'}; t.dim = {3, 3, 3, 3}; t.v.assign(81, 0.0);
    for (int j1 = 0; j1 < 3; ++j1)
      for (int i1 = 0; i1 < 3; ++i1)
        for (int i2 = 0; i2 < 3; ++i2)
          for (int j2 = 0; j2 < 3; ++j2) {
            cd s = 0;
            for (int b = 0; b < 8; ++b) s += TA[b][i1][j1] * TA[b][i2][j2];
            t.v[((j1 * 3 + i1) * 3 + i2) * 3 + j2] = s;
          }
    bc.basis.push_back(t);
  }
  int nl = (int)bc.legs.size();
  int nc = (int)bc.basis.size();
  bc.Ckl.assign(nl * nl, std::vector<cd>(nc * nc, 0.0));
  for (int k = 0; k < nl; ++k)
    for (int l = 0; l < nl; ++l)
      for (int a = 0; a < 8; ++a)
        for (int tau = 0; tau < nc; ++tau) {
          ColTensor t2 = apply_charge(apply_charge(bc.basis[tau], l, a), k, a);
          for (int sig = 0; sig < nc; ++sig) bc.Ckl[k * nl + l][sig * nc + tau] += ct_dot(bc.basis[sig], t2);
        }
}

static BornColour BORNCOL[NPROC];
static bool BORNCOL_DONE[NPROC];
static const BornColour& born_colour(int proc) {
  static std::mutex m;
  std::lock_guard<std::mutex> g(m);
  if (!BORNCOL_DONE[proc]) { build_basis(proc, BORNCOL[proc]); BORNCOL_DONE[proc] = true; }
  return BORNCOL[proc];
}

// Born |M|^2 and colour-linked Borns B_kl (coloured legs, k,l in bc.legs order),
// both including the average factor
static void born_correlations(int proc, const V4* p, Real& B, std::vector<Real>& Bkl) {
  const ProcDef& P = PROCS[proc];
  const BornColour& bc = born_colour(proc);
  const ColourData& c = COLOUR[proc];
  int nl = (int)bc.legs.size();
  int nc = c.nc;
  Bkl.assign(nl * nl, 0.0);
  B = 0;
  std::vector<cd> A(nc);
  Ext ex;
  for (int h = 0; h < (1 << P.npart); ++h) {
    build_ext(proc, p, h, ex, -1, nullptr);
    flows(proc, ex, A.data());
    B += quad(c, A.data());
    for (int q = 0; q < nl * nl; ++q) {
      cd s = 0;
      for (int i = 0; i < nc; ++i)
        for (int j = 0; j < nc; ++j) s += conj(A[i]) * bc.Ckl[q][i * nc + j] * A[j];
      Bkl[q] += s.real();
    }
  }
  B *= P.avg;
  for (auto& x : Bkl) x *= P.avg;
}

// spin-correlated Born: emitter leg's polarisation replaced by the real unit
// vector eperp (eperp.eperp = -1), summed over the other helicities
static Real born_spin_correlated(int proc, const V4* p, int leg, const V4& eperp) {
  const ProcDef& P = PROCS[proc];
  const ColourData& c = COLOUR[proc];
  std::vector<cd> A(c.nc);
  C4 ov = c4(eperp);
  Ext ex;
  Real s = 0;
  int bit = 1 << (P.npart - 1 - leg);
  for (int h = 0; h < (1 << P.npart); ++h) {
    if (h & bit) continue;
    build_ext(proc, p, h, ex, leg, &ov);
    flows(proc, ex, A.data());
    s += quad(c, A.data());
  }
  return s * P.avg;
}

// FKS sector description ----------------------------------------------------
struct FksPair { int i, j; };            // j = -1: initial state (both beams)
struct FksDef {
  int real, born;
  int bornm = -1;                        // Born at the y -> -1 end when it differs (quark FKS parton)
  int nreal, nborn;
  std::vector<FksPair> pairs;            // all FKS pairs of the real process
  std::vector<char> gluon;               // per real leg
  std::vector<char> quark;               // per real leg (massless quark)
};
static FksDef fks_def(int real) {
  FksDef d;
  d.real = real;
  d.nreal = PROCS[real].npart;
  if (real == EE_UUG) { d.born = EE_UU; d.pairs = {{4, 2}, {4, 3}}; }
  else if (real == GG_TTG) { d.born = GG_TT; d.pairs = {{4, -1}}; }
  else if (real == GG_TTGG) { d.born = GG_TTG; d.pairs = {{4, 5}, {5, 4}, {4, -1}, {5, -1}}; }
  else if (real == UU_TTG) { d.born = UU_TT; d.pairs = {{4, -1}}; }
  else if (real == UG_TTU) { d.born = GG_TT; d.bornm = UU_TT; d.pairs = {{4, -1}}; }
  else d.born = -1;
  d.nborn = d.born >= 0 ? PROCS[d.born].npart : 0;
  d.gluon.assign(d.nreal, 0);
  d.quark.assign(d.nreal, 0);
  for (int k = 0; k < d.nreal; ++k) {
    char kind = PROCS[real].kinds[k];
    d.gluon[k] = kind == 'g';
    d.quark[k] = (kind == 'q' || kind == 'Q') && leg_mass(real, k) == 0.0;
  }
  return d;
}

static Real v3dot(const Real* a, const Real* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// polar basis around a unit vector khat: e1 in the (khat, z) plane, e2 = khat x e1
static void perp_basis(const Real* kh, Real* e1, Real* e2) {
  Real st = Sqrt(kh[0] * kh[0] + kh[1] * kh[1]);
  Real ct = kh[2];
  Real cp = st > 0 ? kh[0] / st : 1.0, sp = st > 0 ? kh[1] / st : 0.0;
  e1[0] = ct * cp; e1[1] = ct * sp; e1[2] = -st;
  e2[0] = -sp; e2[1] = cp; e2[2] = 0.0;
}

// boost along unit vector u that multiplies the light-cone component E + p.u
// by rho (and E - p.u by 1/rho); finite also for a massless recoil system
static V4 boost_along(const V4& p, const Real* u, Real rho) {
  Real pl = p.v[1] * u[0] + p.v[2] * u[1] + p.v[3] * u[2];
  Real pp = p.v[0] + pl, pm = p.v[0] - pl;
  Real e2 = 0.5 * (rho * pp + pm / rho);
  Real pl2 = 0.5 * (rho * pp - pm / rho);
  V4 r;
  r.v[0] = e2;
  for (int k = 0; k < 3; ++k) r.v[1 + k] = p.v[1 + k] + (pl2 - pl) * u[k];
  return r;
}
// pure boost taking a vector at rest (mass M) to total momentum K
static V4 boost_to(const V4& p, const V4& K, Real M) {
  Real g = K.v[0] / M;
  Real bp = (K.v[1] * p.v[1] + K.v[2] * p.v[2] + K.v[3] * p.v[3]) / M;   // gamma beta . p
  V4 r;
  r.v[0] = g * p.v[0] + bp;
  Real f = p.v[0] / M + bp / (K.v[0] + M);
  for (int k = 0; k < 3; ++k) r.v[1 + k] = p.v[1 + k] + f * K.v[1 + k];
  return r;
}

// sector function of pair (i, j) at real momenta k (real frame)
static Real sector_value(const FksDef& d, const V4* k, Real sqrt_s, int i, int j) {
  auto xi = [&](int a) { return 2.0 * k[a].v[0] / sqrt_s; };
  auto ycos = [&](int a, int b) {
    Real pa = Sqrt(v3dot(k[a].v + 1, k[a].v + 1)), pb = Sqrt(v3dot(k[b].v + 1, k[b].v + 1));
    return v3dot(k[a].v + 1, k[b].v + 1) / (pa * pb);
  };
  auto term = [&](int a, int b) {
    if (b < 0) {
      Real pa = Sqrt(v3dot(k[a].v + 1, k[a].v + 1));
      Real ya = k[a].v[3] / pa;
      return 1.0 / (xi(a) * (1.0 - ya) * (1.0 + ya));
    }
    Real h = (d.gluon[a] && d.gluon[b]) ? xi(b) / (xi(a) + xi(b)) : 1.0;
    return h / (xi(a) * xi(b) * (1.0 - ycos(a, b)));
  };
  Real num = 0, den = 0;
  for (const FksPair& q : d.pairs) {
    Real t = term(q.i, q.j);
    den += t;
    if (q.i == i && q.j == j) num = t;
  }
  return num / den;
}

// soft limit of the sector function: direction nh of the soft parton i,
// Born momenta kb in Born leg order, bmap[real leg] = Born leg (or -1)
static Real sector_soft(const FksDef& d, const V4* kb, const int* bmap, Real sqrt_s, const Real* nh, int i, int j) {
  Real num = 0, den = 0;
  for (const FksPair& q : d.pairs) {
    if (q.i != i) continue;
    Real t;
    if (q.j < 0) t = 1.0 / ((1.0 - nh[2]) * (1.0 + nh[2]));
    else {
      const V4& pl = kb[bmap[q.j]];
      Real pa = Sqrt(v3dot(pl.v + 1, pl.v + 1));
      Real y = v3dot(nh, pl.v + 1) / pa;
      t = 1.0 / ((2.0 * pl.v[0] / sqrt_s) * (1.0 - y));
    }
    den += t;
    if (q.j == j) num = t;
  }
  return num / den;
}

struct FksOut {
  Real xi, y, gR, gS, gC, gCm, gSC, gSCm, W, me2R, B, S;
  Real jac, dsig;   // xi_max j(xi, y), and the subtracted cross-section density (see below)
};

// The map's phase-space factor j (dPhi_{n+1} = dPhi_n xi j dxi dy dphi) and
// the subtracted cross section per unit Born phase space and per unit
// xi_tilde, y, phi, with j taken at the kinematics of every term:
//   dsig = xi_max / (2 s_B) [j g_R - j(0,y) g_S - j(xi,1) g_C + j(0,1) g_SC] / (xi (1-y))
// Final-state emitter (massless i, j; recoil system of fixed mass): from
//   d3k_i d3k_j / (4 E_i E_j) = (1/4) E_i E_j dE_i dE_j dOmega dy dphi and
//   E_j fixed by the recoil mass, j = s E_j / (64 pi^3 Ebar_j (1 - xi (1-y)/2)),
//   j(0, y) = s / (64 pi^3), j(xi, 1) = z s / (64 pi^3).
// Beams: at fixed real energy d3k_i/(2 E_i (2 pi)^3) dPhi_n(K) gives
//   dPhi_{n+1}(s_R) = s_R xi / (64 pi^3) dxi dy dphi dPhi_n(s_R (1-xi)); with the
//   real flux 1/(2 s_R) and x_1 x_2 = xbar_1 xbar_2 / (1-xi) at fixed Born
//   kinematics this is j = s_B / (64 pi^3 (1-xi)) against the Born flux, and
//   j(0, y) = s_B / (64 pi^3).
static void fks_density(FksOut& o, bool final_state, Real sb, Real xmax, Real jr, Real z) {
  const Real j0 = sb / (64 * PI * PI * PI);
  const Real xi = o.xi, y = o.y;
  Real num;
  if (final_state) {
    num = (jr * o.gR - j0 * o.gS - z * j0 * o.gC + j0 * o.gSC) / (xi * (1 - y));
  } else {
    num = (jr * (o.gR - (1 + y) / 2 * o.gC - (1 - y) / 2 * o.gCm)
           - j0 * (o.gS - (1 + y) / 2 * o.gSC - (1 - y) / 2 * o.gSCm)) / (xi * (1 - y) * (1 + y));
  }
  o.jac = xmax * jr;
  o.dsig = xmax * num / (2 * sb);
}

// one event of the FKS-subtracted real emission for pair (i, j)
static FksOut fks_event(const FksDef& d, int i, int j, const V4* kb_in, Real xit, Real y, Real phi, V4* kreal,
                        bool map_only = false) {
  // The Born point is on shell and conserves momentum by definition.  An
  // input rounded to double does neither exactly (at the 1e-16 level), and
  // the real emission meets its counterterms only as closely as it does: a
  // term of that size over xi (1-y) would remain in W.  So the final-state
  // three-momenta are shifted by a common amount to sum to zero, every
  // energy is put on its mass shell, and the beams (along +-z in the
  // partonic frame) carry half the total energy each.
  V4 kb[8];
  const int nf = d.nborn - 2;
  Real res[3] = {0, 0, 0};
  for (int k = 2; k < d.nborn; ++k)
    for (int m = 0; m < 3; ++m) res[m] += kb_in[k].v[1 + m];
  Real etot = 0;
  for (int k = 2; k < d.nborn; ++k) {
    for (int m = 0; m < 3; ++m) kb[k].v[1 + m] = kb_in[k].v[1 + m] - res[m] / nf;
    const Real m = leg_mass(d.born, k);
    kb[k].v[0] = Sqrt(v3dot(kb[k].v + 1, kb[k].v + 1) + m * m);
    etot += kb[k].v[0];
  }
  kb[0] = V4{{etot / 2, 0, 0, etot / 2}};
  kb[1] = V4{{etot / 2, 0, 0, -etot / 2}};
  const Real g2 = 4.0 * PI * g_alpha_s;
  const Real CF = Real(4) / 3, CA = 3;
  FksOut o{};
  o.y = y;
  int nb = d.nborn;
  Real sqs_b = kb[0].v[0] + kb[1].v[0];
  Real sb = sqs_b * sqs_b;
  int bmap[8];                           // real leg -> Born leg (-1 for i)
  Real nh[3];                          // soft direction of i
  V4 eperp{{0, 0, 0, 0}};
  Real s_real, sqs_real;
  if (j >= 0) {
    // ---------------- final-state emitter --------------------------------
    // real legs: Born legs keep their positions; i is the extra leg
    int jb = -1;
    for (int r = 0, b = 0; r < d.nreal; ++r) {
      if (r == i) { bmap[r] = -1; continue; }
      bmap[r] = b++;
      if (r == j) jb = bmap[r];
    }
    const V4& kj = kb[jb];
    V4 q{{sqs_b, 0, 0, 0}};
    V4 krec{{q.v[0] - kj.v[0], -kj.v[1], -kj.v[2], -kj.v[3]}};
    Real mrec2 = dot(krec, krec);
    Real xmax = 1.0 - mrec2 / sb;
    Real xi = xit * xmax;
    Real Ei = 0.5 * xi * sqs_b;
    Real Ej = (sb - mrec2 - 2.0 * sqs_b * Ei) / (2.0 * sqs_b - 2.0 * Ei * (1.0 - y));
    Real kabs = Sqrt(Ei * Ei + Ej * Ej + 2.0 * Ei * Ej * y);
    Real kjabs = Sqrt(v3dot(kj.v + 1, kj.v + 1));
    Real kh[3] = {kj.v[1] / kjabs, kj.v[2] / kjabs, kj.v[3] / kjabs};
    Real e1[3], e2[3];
    perp_basis(kh, e1, e2);
    Real sy = Sqrt((1.0 - y) * (1.0 + y));
    Real cti = (Ei + Ej * y) / kabs, sti = Ej * sy / kabs;
    Real cphi = Cos(phi), sphi = Sin(phi);
    Real ki_dir[3], ep[3];
    for (int m = 0; m < 3; ++m) {
      ep[m] = cphi * e1[m] + sphi * e2[m];
      ki_dir[m] = cti * kh[m] + sti * ep[m];
      nh[m] = y * kh[m] + sy * ep[m];
    }
    V4 ki{{Ei, Ei * ki_dir[0], Ei * ki_dir[1], Ei * ki_dir[2]}};
    V4 kjn{{Ej, kabs * kh[0] - ki.v[1], kabs * kh[1] - ki.v[2], kabs * kh[2] - ki.v[3]}};
    Real u[3] = {-kh[0], -kh[1], -kh[2]};
    // recoil system along u = -khat: light-cone component (E + |p|) scaled from
    // (sqrt(s) - Ebar_j + |kbar_j|) to (sqrt(s) - E_i - E_j + |k|)
    Real dyr = (sqs_b - Ei - Ej + kabs) / (sqs_b - kj.v[0] + kjabs);
    for (int r = 0; r < d.nreal; ++r) {
      if (r == i) kreal[r] = ki;
      else if (r == j) kreal[r] = kjn;
      else if (r < 2) kreal[r] = kb[bmap[r]];
      else kreal[r] = boost_along(kb[bmap[r]], u, dyr);
    }
    s_real = sb; sqs_real = sqs_b;
    o.xi = xi;
    eperp = V4{{0, ep[0], ep[1], ep[2]}};
    const Real jr = sb / (64 * PI * PI * PI) * (Ej / kj.v[0]) / (1 - xi * (1 - y) / 2);
    if (map_only) {
      o.jac = xmax * jr;
      return o;
    }
    // real matrix element and sector function
    o.me2R = me2_event(d.real, kreal, nullptr);
    o.S = sector_value(d, kreal, sqs_real, i, j);
    o.gR = xi * xi * (1.0 - y) * o.me2R * o.S;
    // Born correlations at the Born kinematics
    Real B;
    std::vector<Real> Bkl;
    born_correlations(d.born, kb, B, Bkl);
    o.B = B;
    const BornColour& bc = born_colour(d.born);
    int nl = (int)bc.legs.size();
    // eikonal: -sum_{kl} (p_k.p_l)/((p_k.n)(p_l.n)) B_kl with n = (1, nh)
    V4 n{{1.0, nh[0], nh[1], nh[2]}};
    Real eik = 0;
    for (int a = 0; a < nl; ++a)
      for (int b = 0; b < nl; ++b) {
        const V4 &pa = kb[bc.legs[a]], &pb = kb[bc.legs[b]];
        eik -= dot(pa, pb) / (dot(pa, n) * dot(pb, n)) * Bkl[a * nl + b];
      }
    Real Ss = sector_soft(d, kb, bmap, sqs_b, nh, i, j);
    o.gS = (1.0 - y) * 4.0 / sb * g2 * eik * Ss;
    // collinear limit y -> 1: E_j^c = Ebar_j - E_i, z = E_j^c / Ebar_j
    Real Ejc = kj.v[0] - Ei;
    Real z = Ejc / kj.v[0];
    Real Sc = (d.gluon[i] && d.gluon[j]) ? z : 1.0;
    Real P;
    Real Cj;
    if (d.gluon[j]) {
      Real Bp = born_spin_correlated(d.born, kb, jb, eperp);
      P = 2.0 * CA * ((z / (1.0 - z) + (1.0 - z) / z) * B + 2.0 * z * (1.0 - z) * Bp);
      Cj = CA;
    } else {
      P = CF * (1.0 + z * z) / (1.0 - z) * B;
      Cj = CF;
    }
    o.gC = 2.0 * xi * g2 / (sqs_b * Ejc) * P * Sc;
    o.gSC = 8.0 * g2 * Cj / sb * B;
    o.W = (o.gR - o.gS - o.gC + o.gSC) / (xi * (1.0 - y));
    fks_density(o, true, sb, xmax, jr, z);
  } else {
    // ---------------- initial-state emitter (both beams) ------------------
    for (int r = 0, b = 0; r < d.nreal; ++r) {
      if (r == i) { bmap[r] = -1; continue; }
      bmap[r] = b++;
    }
    Real xmax = 1.0 - sb / (FKS_SQRT_SCAP * FKS_SQRT_SCAP);
    Real xi = xit * xmax;
    Real sr = sb / (1.0 - xi);
    Real sqr = Sqrt(sr);
    Real Ei = 0.5 * xi * sqr;
    Real sy = Sqrt((1.0 - y) * (1.0 + y));
    Real cphi = Cos(phi), sphi = Sin(phi);
    nh[0] = sy * cphi; nh[1] = sy * sphi; nh[2] = y;
    V4 p1{{0.5 * sqr, 0, 0, 0.5 * sqr}}, p2{{0.5 * sqr, 0, 0, -0.5 * sqr}};
    V4 ki{{Ei, Ei * nh[0], Ei * nh[1], Ei * nh[2]}};
    V4 K{{sqr - Ei, -ki.v[1], -ki.v[2], -ki.v[3]}};
    for (int r = 0; r < d.nreal; ++r) {
      if (r == 0) kreal[r] = p1;
      else if (r == 1) kreal[r] = p2;
      else if (r == i) kreal[r] = ki;
      else kreal[r] = boost_to(kb[bmap[r]], K, sqs_b);
    }
    s_real = sr; sqs_real = sqr;
    o.xi = xi;
    eperp = V4{{0, cphi, sphi, 0}};
    if (map_only) {
      o.jac = xmax * sb / (64 * PI * PI * PI) / (1 - xi);
      return o;
    }
    o.me2R = me2_event(d.real, kreal, nullptr);
    o.S = sector_value(d, kreal, sqs_real, i, -1);
    o.gR = xi * xi * (1.0 - y) * (1.0 + y) * o.me2R * o.S;
    if (d.bornm >= 0) {
      // The FKS parton is a quark (u g -> t tbar u, i = the final u): a soft
      // quark is not singular (g_S = g_SC = 0), and each collinear end changes
      // the flavour of the parton entering the hard process.
      //   y -> +1: u(beam 1) -> u(final) + g(x p1); Born g g -> t tbar;
      //            P_gq with its spin correlation, C_F [x B + 4 (1-x)/x B_perp]
      //   y -> -1: g(beam 2) -> u(final) + ubar(x p2); Born u ubar -> t tbar;
      //            P_qg = T_R [x^2 + (1-x)^2] B
      // Real and Born are both averaged over their own initial spins and
      // colours, so the unpolarised splitting functions apply as they stand
      // (they are defined for averaged initial states); a ratio of spin x
      // colour states n_q/n_g belongs only to raw, unaveraged sums.
      const Real TR = 0.5;
      Real x = 1.0 - xi;
      Real Bplus = me2_event(d.born, kb, nullptr);
      Real Bperp = born_spin_correlated(d.born, kb, 0, eperp);
      Real Bminus = me2_event(d.bornm, kb, nullptr);
      Real Pp = CF * (x * Bplus + 4.0 * (1.0 - x) / x * Bperp);
      Real Pm = TR * (x * x + (1.0 - x) * (1.0 - x)) * Bminus;
      o.B = Bplus;
      o.gS = 0.0;
      o.gC = 8.0 * xi * g2 / sb * Pp;
      o.gCm = 8.0 * xi * g2 / sb * Pm;
      o.gSC = 0.0;
      o.gSCm = 0.0;
      o.W = (o.gR - 0.5 * (1.0 + y) * o.gC - 0.5 * (1.0 - y) * o.gCm) / (xi * (1.0 - y) * (1.0 + y));
      fks_density(o, false, sb, xmax, sb / (64 * PI * PI * PI) / (1 - xi), 0);
      return o;
    }
    Real B;
    std::vector<Real> Bkl;
    born_correlations(d.born, kb, B, Bkl);
    o.B = B;
    const BornColour& bc = born_colour(d.born);
    int nl = (int)bc.legs.size();
    V4 n{{1.0, nh[0], nh[1], nh[2]}};
    Real eik = 0;
    for (int a = 0; a < nl; ++a)
      for (int b = 0; b < nl; ++b) {
        const V4 &pa = kb[bc.legs[a]], &pb = kb[bc.legs[b]];
        eik -= dot(pa, pb) / (dot(pa, n) * dot(pb, n)) * Bkl[a * nl + b];
      }
    Real Ss = sector_soft(d, kb, bmap, sqs_b, nh, i, -1);
    o.gS = (1.0 - y) * (1.0 + y) * 4.0 / sb * g2 * eik * Ss;
    // collinear limits y -> +1 (beam 1) and y -> -1 (beam 2), x = 1 - xi
    Real x = 1.0 - xi;
    Real gc[2], gsc[2];
    for (int side = 0; side < 2; ++side) {
      int beam = side;                           // Born leg of the incoming parton
      Real P, Ca;
      if (d.gluon[beam]) {
        Real Bp = born_spin_correlated(d.born, kb, beam, eperp);
        P = 2.0 * CA * ((x / (1.0 - x) + x * (1.0 - x)) * B + 2.0 * (1.0 - x) / x * Bp);
        Ca = CA;
      } else {
        P = CF * (1.0 + x * x) / (1.0 - x) * B;
        Ca = CF;
      }
      gc[side] = 8.0 * xi * g2 / sb * P;          // S^coll = 1
      gsc[side] = 16.0 * g2 * Ca / sb * B;
    }
    o.gC = gc[0]; o.gCm = gc[1]; o.gSC = gsc[0]; o.gSCm = gsc[1];
    o.W = (o.gR - o.gS - 0.5 * (1.0 + y) * (o.gC - o.gSC) - 0.5 * (1.0 - y) * (o.gCm - o.gSCm))
          / (xi * (1.0 - y) * (1.0 + y));
    fks_density(o, false, sb, xmax, sb / (64 * PI * PI * PI) / (1 - xi), 0);
  }
  (void)s_real;
  return o;
}

extern "C" {

// FKS-subtracted real emission.  real_proc in {ee_uug, gg_ttg, gg_ttgg, uu_ttg, ug_ttu};
// (i, j) an FKS pair of that process (j = -1: initial state).  born_mom: SoA
// [nborn][4][n]; xi_tilde, y, phi: [n].  out: [n][14] = xi, y, g_R, g_S, g_C,
// g_Cm, g_SC, g_SCm, W, |M_R|^2, B, S, jac, dsig.  real_out (optional): SoA [nreal][4][n].
int orc_fks(int real_proc, int i, int j, int64_t n, const double* born_mom, const double* xit, const double* y,
            const double* phi, double* out, double* real_out, int nthreads) {
  init_colour();
  FksDef d = fks_def(real_proc);
  if (d.born < 0) return 1;
  bool ok = false;
  for (const FksPair& q : d.pairs) if (q.i == i && q.j == j) ok = true;
  if (!ok) return 2;
  born_colour(d.born);
  parallel_for(n, nthreads, [&](int64_t e) {
    V4 kb[8], kr[8];
    load_event(born_mom, n, e, d.nborn, kb);
    FksOut o = fks_event(d, i, j, kb, xit[e], y[e], phi[e], kr);
    double* r = out + e * 14;
    r[0] = o.xi; r[1] = o.y; r[2] = o.gR; r[3] = o.gS; r[4] = o.gC; r[5] = o.gCm; r[6] = o.gSC; r[7] = o.gSCm;
    r[8] = o.W; r[9] = o.me2R; r[10] = o.B; r[11] = o.S; r[12] = o.jac; r[13] = o.dsig;
    if (real_out)
      for (int k = 0; k < d.nreal; ++k)
        for (int m = 0; m < 4; ++m) real_out[(k * 4 + m) * n + e] = kr[k].v[m];
  });
  return 0;
}

// The FKS map alone (no matrix elements): out [n][2] = xi, jac (as in
// orc_fks), real_out SoA [nreal][4][n].
int orc_fks_map(int real_proc, int i, int j, int64_t n, const double* born_mom, const double* xit, const double* y,
                const double* phi, double* out, double* real_out, int nthreads) {
  FksDef d = fks_def(real_proc);
  if (d.born < 0) return 1;
  bool ok = false;
  for (const FksPair& q : d.pairs) if (q.i == i && q.j == j) ok = true;
  if (!ok) return 2;
  parallel_for(n, nthreads, [&](int64_t e) {
    V4 kb[8], kr[8];
    load_event(born_mom, n, e, d.nborn, kb);
    FksOut o = fks_event(d, i, j, kb, xit[e], y[e], phi[e], kr, true);
    out[e * 2] = o.xi;
    out[e * 2 + 1] = o.jac;
    if (real_out)
      for (int k = 0; k < d.nreal; ++k)
        for (int m = 0; m < 4; ++m) real_out[(k * 4 + m) * n + e] = kr[k].v[m];
  });
  return 0;
}

// colour-linked Borns B_kl for a Born process (legs in process order of its
// coloured legs): out [n][nl*nl], plus B [n]
int orc_born_correlations(int proc, int64_t n, const double* mom, double* B, double* Bkl, int* nl_out) {
  init_colour();
  if (proc != EE_UU && proc != GG_TT && proc != GG_TTG && proc != UU_TT) return 1;
  const BornColour& bc = born_colour(proc);
  int nl = (int)bc.legs.size();
  *nl_out = nl;
  if (n == 0) return 0;
  parallel_for(n, 8, [&](int64_t e) {
    V4 p[8];
    load_event(mom, n, e, PROCS[proc].npart, p);
    Real b;
    std::vector<Real> kl;
    born_correlations(proc, p, b, kl);
    B[e] = b;
    for (int q = 0; q < nl * nl; ++q) Bkl[e * nl * nl + q] = kl[q];
  });
  return 0;
}

}  // extern "C"

extern "C" {
// every sector function of the real process at real momenta (SoA [nreal][4][n]):
// out [n][npairs] in the order of the process's FKS pairs
int orc_sector_functions(int real_proc, int64_t n, const double* real_mom, double* out, int* npairs) {
  FksDef d = fks_def(real_proc);
  if (d.born < 0) return 1;
  *npairs = (int)d.pairs.size();
  for (int64_t e = 0; e < n; ++e) {
    V4 k[8];
    load_event(real_mom, n, e, d.nreal, k);
    Real sq = k[0].v[0] + k[1].v[0];
    for (size_t q = 0; q < d.pairs.size(); ++q) out[e * d.pairs.size() + q] = sector_value(d, k, sq, d.pairs[q].i, d.pairs[q].j);
  }
  return 0;
}

// spin-correlated Born of a Born process with leg `leg`'s polarisation replaced
// by the real vector eperp (4 doubles, upper index) -- per event, SoA momenta
int orc_born_spin_correlated(int proc, int64_t n, const double* mom, int leg, const double* eperp, double* out) {
  init_colour();
  for (int64_t e = 0; e < n; ++e) {
    V4 p[8];
    load_event(mom, n, e, PROCS[proc].npart, p);
    V4 ev{{eperp[4 * e], eperp[4 * e + 1], eperp[4 * e + 2], eperp[4 * e + 3]}};
    out[e] = born_spin_correlated(proc, p, leg, ev);
  }
  return 0;
}
}

// ============================================================================
// RAMBO phase space (ORACLE) -- Kleiss, Stirling and Ellis's democratic
// generator: n massless momenta drawn isotropically with energy density
// q0 exp(-q0), brought to total momentum (sqrt_s, 0) by one conformal
// (boost + scale) transformation; massive final states by a common rescaling
// of the three-momenta solved for energy conservation (Newton).  The
// uniforms are inputs (four per particle: cos theta, phi, and two for the
// energy), so this checks the arithmetic alone.  After the conformal step a
// projection removes the rounding it leaves (residual three-momentum, E = |p|),
// as the input recipe of the batches does.
// ============================================================================
extern "C" {

int orc_rambo(int nfin, const double* masses, int64_t n, const double* sqrt_s, const double* u, double* p_out,
              double* w_out) {
  if (nfin < 2 || nfin > 8) return 1;
  Real vol1 = Pow(2.0 * PI, 4 - 3 * nfin) * Pow(PI / 2.0, nfin - 1);
  for (int k = 2; k <= nfin - 1; ++k) vol1 /= k;     // 1/(n-1)!
  for (int k = 2; k <= nfin - 2; ++k) vol1 /= k;     // 1/(n-2)!
  bool massive = false;
  Real msum = 0.0;
  for (int i = 0; i < nfin; ++i) { massive = massive || masses[i] > 0.0; msum += masses[i]; }
  for (int64_t e = 0; e < n; ++e) {
    const Real rs = sqrt_s[e];
    const double* ue = u + e * nfin * 4;
    Real q[8][4], Q[4] = {0, 0, 0, 0};
    for (int i = 0; i < nfin; ++i) {
      const Real c = 2.0 * ue[4 * i] - 1.0, ph = 2.0 * PI * ue[4 * i + 1];
      const Real e0 = -Log(ue[4 * i + 2] * ue[4 * i + 3]);
      const Real s = Sqrt(std::max<Real>(0.0, 1.0 - c * c));
      q[i][0] = e0; q[i][1] = e0 * s * Cos(ph); q[i][2] = e0 * s * Sin(ph); q[i][3] = e0 * c;
      for (int m = 0; m < 4; ++m) Q[m] += q[i][m];
    }
    // conformal transformation: boost by -Q/M, scale by sqrt_s/M
    const Real M = Sqrt(Q[0] * Q[0] - Q[1] * Q[1] - Q[2] * Q[2] - Q[3] * Q[3]);
    const Real b[3] = {-Q[1] / M, -Q[2] / M, -Q[3] / M};
    const Real g = Q[0] / M, a = 1.0 / (1.0 + g), x = rs / M;
    Real p[8][4];
    for (int i = 0; i < nfin; ++i) {
      const Real bq = b[0] * q[i][1] + b[1] * q[i][2] + b[2] * q[i][3];
      p[i][0] = x * (g * q[i][0] + bq);
      for (int m = 0; m < 3; ++m) p[i][1 + m] = x * (q[i][1 + m] + b[m] * q[i][0] + a * bq * b[m]);
    }
    // projection of the rounding left by the transformation
    Real r3[3] = {0, 0, 0};
    for (int i = 0; i < nfin; ++i) for (int m = 0; m < 3; ++m) r3[m] += p[i][1 + m];
    Real pabs[8], tot = 0.0;
    for (int i = 0; i < nfin; ++i) {
      for (int m = 0; m < 3; ++m) p[i][1 + m] -= r3[m] / nfin;
      pabs[i] = Sqrt(p[i][1] * p[i][1] + p[i][2] * p[i][2] + p[i][3] * p[i][3]);
      tot += pabs[i];
    }
    const Real sc = rs / tot;
    for (int i = 0; i < nfin; ++i) {
      for (int m = 0; m < 3; ++m) p[i][1 + m] *= sc;
      p[i][0] = pabs[i] * sc;
    }
    Real w = vol1 * Pow(rs, 2 * (nfin - 2));
    if (massive) {
      // common factor xi on the three-momenta: sum_i sqrt(m_i^2 + xi^2 E_i^2) = sqrt_s
      Real xi = Sqrt(std::max<Real>(1e-30, 1.0 - (msum / rs) * (msum / rs)));
      for (int it = 0; it < 50; ++it) {
        Real f = -rs, fp = 0.0;
        for (int i = 0; i < nfin; ++i) {
          const Real ek = Sqrt(masses[i] * masses[i] + xi * xi * p[i][0] * p[i][0]);
          f += ek;
          fp += xi * p[i][0] * p[i][0] / ek;
        }
        xi -= f / fp;
        if (Fabs(f) <= 1e-14 * rs) break;
      }
      Real ksum = 0.0, kprod = 1.0, k2e = 0.0;
      for (int i = 0; i < nfin; ++i) {
        const Real E = p[i][0];
        const Real k0 = Sqrt(masses[i] * masses[i] + xi * xi * E * E);
        for (int m = 0; m < 3; ++m) p[i][1 + m] *= xi;
        p[i][0] = k0;
        const Real ka = Sqrt(p[i][1] * p[i][1] + p[i][2] * p[i][2] + p[i][3] * p[i][3]);
        ksum += ka; kprod *= ka / k0; k2e += ka * ka / k0;
      }
      w *= Pow(ksum / rs, 2 * nfin - 3) * kprod * rs / k2e;
    }
    for (int i = 0; i < nfin; ++i) for (int m = 0; m < 4; ++m) p_out[(e * nfin + i) * 4 + m] = p[i][m];
    w_out[e] = w;
  }
  return 0;
}

}  // extern "C"
