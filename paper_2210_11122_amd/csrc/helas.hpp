// helas.hpp -- per-lane wavefunction algebra for the tree-level matrix-element kernels.
//
// One lane holds one (event, helicity) pair.  Wavefunctions are four complex components
// (a Dirac spinor in the chiral representation, or a contravariant Lorentz vector) in the
// real type R: double for the FP64 kernels, float for the mixed-precision kernels.
// Momenta, propagator denominators and momentum sums are always double; in the mixed form
// they are rounded to float only where they multiply a wavefunction.
//
// Conventions (the standard LO Feynman rules in Feynman gauge, metric (+,-,-,-)):
//   quark-gluon vertex  i g gamma^mu (colour t^a stripped)
//   quark propagator    i (qslash + m) / (q^2 - m^2)
//   gluon propagator    -i g_{mu nu} / P^2
//   three-gluon vertex  g [g^{mu nu}(k-p)^rho + g^{nu rho}(p-q)^mu + g^{rho mu}(q-k)^nu]
//                       (colour f^{abc} stripped, all momenta incoming)
//   four-gluon vertex   -i g^2 x (one of its three Lorentz structures; colour f f stripped)
// External states are helicity eigenstates with the HELAS phase conventions (Hagiwara,
// Murayama, Watanabe, KEK-91-11): u(p,l) = (w_{-l} chi_l, w_l chi_l),
// v(p,l) = (-l w_l chi_{-l}, l w_{-l} chi_{-l}), w_pm = sqrt(E pm |p|), and
// eps(k,l) = (-l e1 - i e2)/sqrt(2) (complex conjugate for an outgoing gluon).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace me {

template <class R>
struct cx {
    R r, i;
};

template <class R>
__device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.r + b.r, a.i + b.i}; }
template <class R>
__device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.r - b.r, a.i - b.i}; }
template <class R>
__device__ __forceinline__ cx<R> operator*(cx<R> a, cx<R> b)
{
    return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r};
}
template <class R>
__device__ __forceinline__ cx<R> operator*(R s, cx<R> a) { return {s * a.r, s * a.i}; }
// i * a
template <class R>
__device__ __forceinline__ cx<R> mul_i(cx<R> a) { return {-a.i, a.r}; }
// c + a b and c - a b as chains of fused multiply-adds (4 instead of 2 mul + 2 fma + 2 add)
template <class R>
__device__ __forceinline__ cx<R> cfma(cx<R> a, cx<R> b, cx<R> c)
{
    return {fma(a.r, b.r, fma(-a.i, b.i, c.r)), fma(a.r, b.i, fma(a.i, b.r, c.i))};
}
template <class R>
__device__ __forceinline__ cx<R> cfms(cx<R> a, cx<R> b, cx<R> c)
{
    return {fma(-a.r, b.r, fma(a.i, b.i, c.r)), fma(-a.r, b.i, fma(-a.i, b.r, c.i))};
}

struct P4 {
    double t, x, y, z;
};
__device__ __forceinline__ P4 operator+(const P4& a, const P4& b)
{
    return {a.t + b.t, a.x + b.x, a.y + b.y, a.z + b.z};
}
__device__ __forceinline__ P4 operator-(const P4& a, const P4& b)
{
    return {a.t - b.t, a.x - b.x, a.y - b.y, a.z - b.z};
}
__device__ __forceinline__ P4 operator-(const P4& a) { return {-a.t, -a.x, -a.y, -a.z}; }
__device__ __forceinline__ double msq(const P4& a) { return a.t * a.t - a.x * a.x - a.y * a.y - a.z * a.z; }

// 1/x and 1/sqrt(x) in double: the hardware estimate refined by two Newton steps (within
// an ulp or two of the correctly rounded result, without the IEEE division sequence)
__device__ __forceinline__ double rcp(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}
__device__ __forceinline__ double rsqrt_nr(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    double h = 0.5 * x;
    y = y * __builtin_fma(-h * y, y, 1.5);
    return y * __builtin_fma(-h * y, y, 1.5);
}

template <class R>
struct W4 {
    cx<R> c[4];
};

// Minkowski product of two complex vectors (no conjugation)
template <class R>
__device__ __forceinline__ cx<R> dot(const W4<R>& a, const W4<R>& b)
{
    return cfms(a.c[3], b.c[3], cfms(a.c[2], b.c[2], cfms(a.c[1], b.c[1], a.c[0] * b.c[0])));
}
// x + u y for a unit u = UR + i UI of the Gaussian integers (1, -1, i or -i): the vertices are
// linear in each wavefunction, so amplitudes that differ in one operand only sum before the vertex
template <class R, int UR, int UI>
__device__ __forceinline__ W4<R> w4_acc(const W4<R>& x, const W4<R>& y)
{
    static_assert(UR * UR + UI * UI == 1, "a unit of the Gaussian integers");
    W4<R> o;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        if (UR == 1) o.c[mu] = x.c[mu] + y.c[mu];
        else if (UR == -1) o.c[mu] = x.c[mu] - y.c[mu];
        else if (UI == 1) o.c[mu] = x.c[mu] + mul_i(y.c[mu]);
        else o.c[mu] = x.c[mu] - mul_i(y.c[mu]);
    }
    return o;
}
// real vector in the working precision
template <class R>
struct R4 {
    R t, x, y, z;
};
template <class R>
__device__ __forceinline__ R4<R> rnd(const P4& p) { return {(R)p.t, (R)p.x, (R)p.y, (R)p.z}; }
template <class R>
__device__ __forceinline__ cx<R> dot(const W4<R>& a, const R4<R>& k)
{
    return {a.c[0].r * k.t - a.c[1].r * k.x - a.c[2].r * k.y - a.c[3].r * k.z,
            a.c[0].i * k.t - a.c[1].i * k.x - a.c[2].i * k.y - a.c[3].i * k.z};
}

// ------------------------------------------------------------------------------------
// external states (computed in double, rounded to R)

// two-component helicity eigenstates of sigma.p/|p|; (0,1) / (-1,0) for p along -z
__device__ __forceinline__ void chi2(const P4& p, int lam, double out[4])
{
    double pp2 = p.x * p.x + p.y * p.y + p.z * p.z;
    double pp = pp2 * rsqrt_nr(pp2);
    double d = (p.z >= 0.0) ? pp + p.z : (p.x * p.x + p.y * p.y) * rcp(pp - p.z);
    if (!(d > 0.0)) {
        if (lam > 0) { out[0] = 0; out[1] = 0; out[2] = 1; out[3] = 0; }
        else { out[0] = -1; out[1] = 0; out[2] = 0; out[3] = 0; }
        return;
    }
    double nrm = rsqrt_nr(2.0 * pp * d);
    if (lam > 0) { out[0] = d * nrm; out[1] = 0; out[2] = p.x * nrm; out[3] = p.y * nrm; }
    else { out[0] = -p.x * nrm; out[1] = p.y * nrm; out[2] = d * nrm; out[3] = 0; }
}

// u(p, lam) as a row ubar = u^dagger gamma^0 = (u2*, u3*, u0*, u1*)
template <class R>
__device__ __forceinline__ W4<R> ext_ubar(const P4& p, double m, int lam)
{
    double c[4];
    chi2(p, lam, c);
    double ep = p.t + sqrt(p.x * p.x + p.y * p.y + p.z * p.z), iw = rsqrt_nr(ep);
    double wp = ep * iw, wm = m * iw;
    double up = lam > 0 ? wm : wp, lo = lam > 0 ? wp : wm;
    W4<R> w;
    w.c[0] = {(R)(lo * c[0]), (R)(-lo * c[1])};
    w.c[1] = {(R)(lo * c[2]), (R)(-lo * c[3])};
    w.c[2] = {(R)(up * c[0]), (R)(-up * c[1])};
    w.c[3] = {(R)(up * c[2]), (R)(-up * c[3])};
    return w;
}
// u(p, lam) as a column
template <class R>
__device__ __forceinline__ W4<R> ext_u(const P4& p, double m, int lam)
{
    double c[4];
    chi2(p, lam, c);
    double ep = p.t + sqrt(p.x * p.x + p.y * p.y + p.z * p.z), iw = rsqrt_nr(ep);
    double wp = ep * iw, wm = m * iw;
    double up = lam > 0 ? wm : wp, lo = lam > 0 ? wp : wm;
    W4<R> w;
    w.c[0] = {(R)(up * c[0]), (R)(up * c[1])};
    w.c[1] = {(R)(up * c[2]), (R)(up * c[3])};
    w.c[2] = {(R)(lo * c[0]), (R)(lo * c[1])};
    w.c[3] = {(R)(lo * c[2]), (R)(lo * c[3])};
    return w;
}
// v(p, lam) as a column
template <class R>
__device__ __forceinline__ W4<R> ext_v(const P4& p, double m, int lam)
{
    double c[4];
    chi2(p, -lam, c);
    double ep = p.t + sqrt(p.x * p.x + p.y * p.y + p.z * p.z), iw = rsqrt_nr(ep);
    double wp = ep * iw, wm = m * iw;
    double wl = lam > 0 ? wp : wm, wml = lam > 0 ? wm : wp;
    double up = -lam * wl, lo = lam * wml;
    W4<R> w;
    w.c[0] = {(R)(up * c[0]), (R)(up * c[1])};
    w.c[1] = {(R)(up * c[2]), (R)(up * c[3])};
    w.c[2] = {(R)(lo * c[0]), (R)(lo * c[1])};
    w.c[3] = {(R)(lo * c[2]), (R)(lo * c[3])};
    return w;
}
// v(p, lam) as a row vbar = v^dagger gamma^0
template <class R>
__device__ __forceinline__ W4<R> ext_vbar(const P4& p, double m, int lam)
{
    W4<R> v = ext_v<R>(p, m, lam);
    W4<R> w;
    w.c[0] = {v.c[2].r, -v.c[2].i};
    w.c[1] = {v.c[3].r, -v.c[3].i};
    w.c[2] = {v.c[0].r, -v.c[0].i};
    w.c[3] = {v.c[1].r, -v.c[1].i};
    return w;
}
// The polarisation vectors of a massless vector boson are fixed by five numbers of its
// direction (theta, phi), r = 1/sqrt(2):
//   a = r cos(theta) cos(phi), b = r cos(theta) sin(phi), c = r sin(theta),
//   d = r sin(phi), e = r cos(phi)
// (along +-z: phi = 0).  The helicity and the conjugation of an outgoing boson only flip signs.
template <class T>
struct GBT {
    T a, b, c, d, e;
};
typedef GBT<double> GB;
__device__ __forceinline__ GB gluon_basis(const P4& k)
{
    double kt2 = k.x * k.x + k.y * k.y;
    double ikk = rsqrt_nr(kt2 + k.z * k.z);
    double ct = k.z * ikk, st = 0.0, cp = 1.0, sp = 0.0;
    if (kt2 > 0.0) {
        double ikt = rsqrt_nr(kt2);
        st = kt2 * ikt * ikk;
        cp = k.x * ikt;
        sp = k.y * ikt;
    }
    const double r = 0.70710678118654752440;
    return {r * ct * cp, r * ct * sp, r * st, r * sp, r * cp};
}
// the basis in the working precision (rounding commutes with the sign flips below, so the
// vectors are those of the FP64 basis rounded)
template <class R>
__device__ __forceinline__ GBT<R> gb_cast(const GB& g)
{
    return {(R)g.a, (R)g.b, (R)g.c, (R)g.d, (R)g.e};
}
// polarisation vector of helicity lam from the basis; complex conjugate if outgoing
template <class R>
__device__ __forceinline__ W4<R> ext_vec_b(const GBT<R>& g, int lam, bool outgoing)
{
    const R m = (R)(-lam);   // exact: lam = +-1
    W4<R> w;
    w.c[0] = {(R)0, (R)0};
    w.c[1] = {m * g.a, outgoing ? -g.d : g.d};
    w.c[2] = {m * g.b, outgoing ? g.e : -g.e};
    w.c[3] = {-m * g.c, (R)0};
    return w;
}
// gluon / photon polarisation vector of momentum k; complex conjugate if outgoing (the same
// values as ext_vec_b of gluon_basis(k): the products below differ from those only by signs)
template <class R>
__device__ __forceinline__ W4<R> ext_vec(const P4& k, int lam, bool outgoing)
{
    double kt2 = k.x * k.x + k.y * k.y;
    double ikk = rsqrt_nr(kt2 + k.z * k.z);
    double ct = k.z * ikk, st = 0.0, cp = 1.0, sp = 0.0;
    if (kt2 > 0.0) {
        double ikt = rsqrt_nr(kt2);
        st = kt2 * ikt * ikk;
        cp = k.x * ikt;
        sp = k.y * ikt;
    }
    const double r = 0.70710678118654752440;
    const double s = outgoing ? -r : r;
    W4<R> w;
    w.c[0] = {(R)0, (R)0};
    w.c[1] = {(R)(-lam * r * ct * cp), (R)(s * sp)};
    w.c[2] = {(R)(-lam * r * ct * sp), (R)(-s * cp)};
    w.c[3] = {(R)(lam * r * st), (R)0};
    return w;
}

// ------------------------------------------------------------------------------------
// Dirac algebra in the chiral representation, gamma.G = [[0, G.sigma], [G.sigmabar, 0]]
// with a = G0+G3, b = G0-G3, c = G1+iG2, d = G1-iG2.

// (gamma.G) psi for a column spinor
template <class R>
__device__ __forceinline__ W4<R> gslash_col(const W4<R>& G, const W4<R>& s)
{
    cx<R> a = G.c[0] + G.c[3], b = G.c[0] - G.c[3];
    cx<R> c = G.c[1] + mul_i(G.c[2]), d = G.c[1] - mul_i(G.c[2]);
    W4<R> o;
    o.c[0] = cfms(d, s.c[3], b * s.c[2]);
    o.c[1] = cfms(c, s.c[2], a * s.c[3]);
    o.c[2] = cfma(d, s.c[1], a * s.c[0]);
    o.c[3] = cfma(b, s.c[1], c * s.c[0]);
    return o;
}
// ubar (gamma.G) for a row spinor
template <class R>
__device__ __forceinline__ W4<R> gslash_row(const W4<R>& u, const W4<R>& G)
{
    cx<R> a = G.c[0] + G.c[3], b = G.c[0] - G.c[3];
    cx<R> c = G.c[1] + mul_i(G.c[2]), d = G.c[1] - mul_i(G.c[2]);
    W4<R> o;
    o.c[0] = cfma(u.c[3], c, u.c[2] * a);
    o.c[1] = cfma(u.c[3], b, u.c[2] * d);
    o.c[2] = cfms(u.c[1], c, u.c[0] * b);
    o.c[3] = cfms(u.c[0], d, u.c[1] * a);
    return o;
}
// f (qslash + m) phi for a column spinor and real q
template <class R>
__device__ __forceinline__ W4<R> qslash_col(const R4<R>& q, R m, R f, const W4<R>& s)
{
    R a = q.t + q.z, b = q.t - q.z;
    W4<R> o;
    // c = q1 + i q2, d = q1 - i q2 (complex with real parts)
    cx<R> cs2 = {q.x * s.c[2].r - q.y * s.c[2].i, q.x * s.c[2].i + q.y * s.c[2].r};  // c*s2
    cx<R> ds3 = {q.x * s.c[3].r + q.y * s.c[3].i, q.x * s.c[3].i - q.y * s.c[3].r};  // d*s3
    cx<R> cs0 = {q.x * s.c[0].r - q.y * s.c[0].i, q.x * s.c[0].i + q.y * s.c[0].r};  // c*s0
    cx<R> ds1 = {q.x * s.c[1].r + q.y * s.c[1].i, q.x * s.c[1].i - q.y * s.c[1].r};  // d*s1
    o.c[0] = f * (b * s.c[2] - ds3 + m * s.c[0]);
    o.c[1] = f * (a * s.c[3] - cs2 + m * s.c[1]);
    o.c[2] = f * (a * s.c[0] + ds1 + m * s.c[2]);
    o.c[3] = f * (cs0 + b * s.c[1] + m * s.c[3]);
    return o;
}
// f phibar (qslash + m) for a row spinor and real q
template <class R>
__device__ __forceinline__ W4<R> qslash_row(const R4<R>& q, R m, R f, const W4<R>& u)
{
    R a = q.t + q.z, b = q.t - q.z;
    cx<R> u3c = {q.x * u.c[3].r - q.y * u.c[3].i, q.x * u.c[3].i + q.y * u.c[3].r};  // u3*c
    cx<R> u2d = {q.x * u.c[2].r + q.y * u.c[2].i, q.x * u.c[2].i - q.y * u.c[2].r};  // u2*d
    cx<R> u1c = {q.x * u.c[1].r - q.y * u.c[1].i, q.x * u.c[1].i + q.y * u.c[1].r};  // u1*c
    cx<R> u0d = {q.x * u.c[0].r + q.y * u.c[0].i, q.x * u.c[0].i - q.y * u.c[0].r};  // u0*d
    W4<R> o;
    o.c[0] = f * (a * u.c[2] + u3c + m * u.c[0]);
    o.c[1] = f * (u2d + b * u.c[3] + m * u.c[1]);
    o.c[2] = f * (b * u.c[0] - u1c + m * u.c[2]);
    o.c[3] = f * (a * u.c[1] - u0d + m * u.c[3]);
    return o;
}

// ------------------------------------------------------------------------------------
// currents and amplitudes

// antiquark-side string extended by one vertex: S(q) (i g gamma.G) psi
//   = -g/(q^2-m^2) (qslash + m)(gamma.G) psi
template <class R>
__device__ __forceinline__ W4<R> fstr_v(const W4<R>& psi, const W4<R>& G, const P4& q, double m, double g)
{
    double f = -g * rcp(msq(q) - m * m);
    return qslash_col<R>(rnd<R>(q), (R)m, (R)f, gslash_col<R>(G, psi));
}
// quark-side string extended by one vertex: ubar (i g gamma.G) S(q)
template <class R>
__device__ __forceinline__ W4<R> fstr_u(const W4<R>& ub, const W4<R>& G, const P4& q, double m, double g)
{
    double f = -g * rcp(msq(q) - m * m);
    return qslash_row<R>(rnd<R>(q), (R)m, (R)f, gslash_row<R>(ub, G));
}
// gluon emitted by the pair (ubar, psi): (-i/P^2)(i g ubar gamma^mu psi) = (g/P^2) ubar gamma^mu psi
template <class R>
__device__ __forceinline__ W4<R> jf(const W4<R>& u, const W4<R>& s, const P4& P, double g)
{
    R f = (R)(g * rcp(msq(P)));
    cx<R> u0s2 = u.c[0] * s.c[2], u1s3 = u.c[1] * s.c[3], u2s0 = u.c[2] * s.c[0], u3s1 = u.c[3] * s.c[1];
    cx<R> u0s3 = u.c[0] * s.c[3], u1s2 = u.c[1] * s.c[2], u2s1 = u.c[2] * s.c[1], u3s0 = u.c[3] * s.c[0];
    W4<R> o;
    o.c[0] = f * (u0s2 + u1s3 + u2s0 + u3s1);
    o.c[1] = f * (u0s3 + u1s2 - u2s1 - u3s0);
    o.c[2] = f * mul_i(u1s2 - u0s3 + u2s1 - u3s0);
    o.c[3] = f * (u0s2 - u1s3 - u2s0 + u3s1);
    return o;
}
// three-gluon current with the off-shell leg first: (-i g / P^2) V, P = k1 + k2,
// V = (J1.J2)(k1-k2) + J2 (J1.(k1+2k2)) - J1 (J2.(2k1+k2))
template <class R>
__device__ __forceinline__ W4<R> vvv_cur(const W4<R>& J1, const P4& k1, const W4<R>& J2, const P4& k2, double g)
{
    double f = g * rcp(msq(k1 + k2));
    R4<R> a = rnd<R>(k1 - k2), b = rnd<R>(k1 + k2 + k2), c = rnd<R>(k1 + k1 + k2);
    cx<R> d12 = dot(J1, J2), d1b = dot(J1, b), d2c = dot(J2, c);
    R ar[4] = {a.t, a.x, a.y, a.z};
    W4<R> o;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        cx<R> v = cfms(J1.c[mu], d2c, cfma(J2.c[mu], d1b, ar[mu] * d12));
        o.c[mu] = {(R)f * v.i, -(R)f * v.r};  // -i f v
    }
    return o;
}
// four-gluon current: (-i/P^2)(-i g^2) L = -(g^2/P^2) L with L one of
//   S0: Jb (Ja.Jc) - Jc (Ja.Jb);  S1: Ja (Jb.Jc) - Jc (Ja.Jb);  S2: Ja (Jb.Jc) - Jb (Ja.Jc)
template <class R, int S>
__device__ __forceinline__ W4<R> vvvv_cur(const W4<R>& Ja, const W4<R>& Jb, const W4<R>& Jc, const P4& P, double g)
{
    R f = (R)(-g * g * rcp(msq(P)));
    W4<R> o;
    if (S == 0) {
        cx<R> ac = dot(Ja, Jc), ab = dot(Ja, Jb);
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) o.c[mu] = f * cfms(Jc.c[mu], ab, Jb.c[mu] * ac);
    } else if (S == 1) {
        cx<R> bc = dot(Jb, Jc), ab = dot(Ja, Jb);
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) o.c[mu] = f * cfms(Jc.c[mu], ab, Ja.c[mu] * bc);
    } else {
        cx<R> bc = dot(Jb, Jc), ac = dot(Ja, Jc);
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) o.c[mu] = f * cfms(Jb.c[mu], ac, Ja.c[mu] * bc);
    }
    return o;
}
// amplitude of a quark-gluon vertex: ubar (i g gamma.G) psi
template <class R>
__device__ __forceinline__ cx<R> amp_ffv(const W4<R>& u, const W4<R>& s, const W4<R>& G, double g)
{
    W4<R> t = gslash_col<R>(G, s);
    cx<R> x = cfma(u.c[3], t.c[3], cfma(u.c[2], t.c[2], cfma(u.c[1], t.c[1], u.c[0] * t.c[0])));
    return (R)g * mul_i(x);
}
// Chiral couplings (gamma5 = diag(-1, -1, 1, 1): P_L keeps components 0, 1 of a column spinor).
// Massive vector boson emitted by the pair (ubar, psi) through i gz gamma^mu (cl P_L + cr P_R),
// with the propagator -i g_{mu nu} / (P^2 - M^2 + i M Gamma) (its P_mu P_nu term drops out
// between massless currents): (gz / (P^2 - M^2 + i M Gamma)) ubar gamma^mu (cl P_L + cr P_R) psi
template <class R>
__device__ __forceinline__ W4<R> jf_chiral(const W4<R>& u, const W4<R>& s, const P4& P, double gz, double cl,
                                           double cr, double M, double Gam)
{
    const double dr = msq(P) - M * M, di = M * Gam;
    const double inv = gz * rcp(dr * dr + di * di);
    const cx<R> f = {(R)(dr * inv), (R)(-di * inv)};
    const R L = (R)cl, Rr = (R)cr;
    cx<R> u0s2 = u.c[0] * s.c[2], u1s3 = u.c[1] * s.c[3], u2s0 = u.c[2] * s.c[0], u3s1 = u.c[3] * s.c[1];
    cx<R> u0s3 = u.c[0] * s.c[3], u1s2 = u.c[1] * s.c[2], u2s1 = u.c[2] * s.c[1], u3s0 = u.c[3] * s.c[0];
    W4<R> o;
    o.c[0] = f * (Rr * (u0s2 + u1s3) + L * (u2s0 + u3s1));
    o.c[1] = f * (Rr * (u0s3 + u1s2) - L * (u2s1 + u3s0));
    o.c[2] = f * mul_i(Rr * (u1s2 - u0s3) + L * (u2s1 - u3s0));
    o.c[3] = f * (Rr * (u0s2 - u1s3) + L * (u3s1 - u2s0));
    return o;
}
// amplitude ubar (i gz gamma.G (cl P_L + cr P_R)) psi
template <class R>
__device__ __forceinline__ cx<R> amp_ffv_chiral(const W4<R>& u, const W4<R>& s, const W4<R>& G, double gz,
                                                double cl, double cr)
{
    W4<R> t = gslash_col<R>(G, s);   // t0, t1 come from psi's components 2, 3 (P_R); t2, t3 from 0, 1
    cx<R> x = (R)cr * (u.c[0] * t.c[0] + u.c[1] * t.c[1]) + (R)cl * (u.c[2] * t.c[2] + u.c[3] * t.c[3]);
    return (R)gz * mul_i(x);
}
// amplitude of a three-gluon vertex with legs (x, a, b), incoming momenta kx, ka, kb:
// g [(Wx.Wa)((kx-ka).Wb) + (Wa.Wb)((ka-kb).Wx) + (Wb.Wx)((kb-kx).Wa)]
template <class R>
__device__ __forceinline__ cx<R> amp_vvv(const W4<R>& Wx, const P4& kx, const W4<R>& Wa, const P4& ka,
                                         const W4<R>& Wb, const P4& kb, double g)
{
    cx<R> xa = dot(Wx, Wa), ab = dot(Wa, Wb), bx = dot(Wb, Wx);
    cx<R> t1 = dot(Wb, rnd<R>(kx - ka)), t2 = dot(Wx, rnd<R>(ka - kb)), t3 = dot(Wa, rnd<R>(kb - kx));
    return (R)g * cfma(bx, t3, cfma(ab, t2, xa * t1));
}
// amplitude of a four-gluon vertex, legs (x, a, b, c): -i g^2 times
//   S0: (x.b)(a.c) - (x.c)(a.b);  S1: (x.a)(b.c) - (x.c)(a.b);  S2: (x.a)(b.c) - (x.b)(a.c)
template <class R, int S>
__device__ __forceinline__ cx<R> amp_vvvv(const W4<R>& Wx, const W4<R>& Wa, const W4<R>& Wb, const W4<R>& Wc,
                                          double g)
{
    cx<R> v;
    if (S == 0) v = cfms(dot(Wx, Wc), dot(Wa, Wb), dot(Wx, Wb) * dot(Wa, Wc));
    else if (S == 1) v = cfms(dot(Wx, Wc), dot(Wa, Wb), dot(Wx, Wa) * dot(Wb, Wc));
    else v = cfms(dot(Wx, Wb), dot(Wa, Wc), dot(Wx, Wa) * dot(Wb, Wc));
    cx<R> iv = mul_i(v);
    return (R)(-g * g) * iv;
}

// ------------------------------------------------------------------------------------
// launch helpers

// Workgroups are dealt to the 8 XCDs round-robin; renumber them so that consecutive
// logical workgroup ids (the helicities of one event block) share an XCD and its L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t w, int64_t n)
{
    const int64_t nx = 8;
    int64_t xcd = w % nx, idx = w / nx;
    int64_t per = n / nx, rem = n % nx;
    return (xcd < rem) ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

// Stage the momenta of events [e0, e0+64) (layout [event][particle][4], double) through
// LDS with coalesced 16-byte loads, into component pairs lds2[2 i + (E, px) | (py, pz)][lane]
// (16 bytes per lane, so a lane reads a four-momentum with two conflict-free 16-byte LDS
// loads); lanes past n_evt read zeros.  WG waves of a workgroup (tid = threadIdx.x) share the
// work and the staged block.
template <int NPAR, int WG = 1>
__device__ __forceinline__ void stage_momenta(const double* __restrict__ mom, int64_t n_evt, int64_t e0,
                                              double* lds, int tid)
{
    constexpr int NCOMP = 4 * NPAR;
    constexpr int NLOAD = 64 * NCOMP / 2;  // double2 elements of the block
    const double2* src = reinterpret_cast<const double2*>(mom + e0 * NCOMP);
    const int64_t n_here = (n_evt - e0) < 64 ? (n_evt - e0) : 64;
#pragma unroll
    for (int k = 0; k < (NLOAD + 64 * WG - 1) / (64 * WG); ++k) {
        const int f = tid + 64 * WG * k;  // double2 index within the block
        if (NLOAD % (64 * WG) != 0 && f >= NLOAD) break;
        const int ev = (2 * f) / NCOMP;   // event within the block
        const int c = (2 * f) % NCOMP;    // first component
        double2 v = {0.0, 0.0};
        if (ev < n_here) v = src[f];
        reinterpret_cast<double2*>(lds)[(c / 2) * 64 + ev] = v;   // c is even: one component pair
    }
    __syncthreads();
}

// as stage_momenta, for a workgroup of `threads` threads known only at run time
template <int NPAR>
__device__ __forceinline__ void stage_momenta_n(const double* __restrict__ mom, int64_t n_evt, int64_t e0,
                                                double* lds, int tid, int threads)
{
    constexpr int NCOMP = 4 * NPAR;
    constexpr int NLOAD = 64 * NCOMP / 2;  // double2 elements of the block
    const double2* src = reinterpret_cast<const double2*>(mom + e0 * NCOMP);
    const int64_t n_here = (n_evt - e0) < 64 ? (n_evt - e0) : 64;
    for (int f = tid; f < NLOAD; f += threads) {
        const int ev = (2 * f) / NCOMP;
        const int c = (2 * f) % NCOMP;
        double2 v = {0.0, 0.0};
        if (ev < n_here) v = src[f];
        reinterpret_cast<double2*>(lds)[(c / 2) * 64 + ev] = v;
    }
    __syncthreads();
}

}  // namespace me

namespace me {
// momentum of particle i of this lane's event, re-read from the LDS staging area at every
// use (volatile: the compiler neither caches nor hoists it, so no four-momentum stays live)
__device__ __forceinline__ P4 lds_p4(const double* lds, int i, int lane)
{
    typedef double v2d __attribute__((ext_vector_type(2)));
    typedef __attribute__((address_space(3))) const volatile v2d lds_v2d;
    lds_v2d* v = (lds_v2d*)lds;
    const v2d a = v[(2 * i) * 64 + lane], b = v[(2 * i + 1) * 64 + lane];
    return {a.x, a.y, b.x, b.y};
}
// Gluon bases of the block's events in LDS (shared by every helicity wave of the workgroup),
// in the working precision R, written once after the momenta are staged: for gluon j (particle
// gp[j]) and event ev, three pairs (a, b), (c, d), (e, 0) at gbl[(3 j + q) * 64 + ev].  Programs
// that keep no external gluon wavefunction in registers rebuild it from here at each use.
template <class R, int NGL, int WG>
__device__ __forceinline__ void stage_gluon_basis(const double* lds, R* gbl, const int (&gp)[NGL], int tid)
{
    typedef R v2 __attribute__((ext_vector_type(2)));
    v2* g2 = reinterpret_cast<v2*>(gbl);
    const int wave = tid >> 6, ev = tid & 63;
#pragma unroll
    for (int j = 0; j < NGL; ++j) {  // gluon j by wave j % WG, one event per lane
        if (j % WG != wave) continue;
        const GBT<R> g = gb_cast<R>(gluon_basis(lds_p4(lds, gp[j], ev)));
        g2[(3 * j) * 64 + ev] = {g.a, g.b};
        g2[(3 * j + 1) * 64 + ev] = {g.c, g.d};
        g2[(3 * j + 2) * 64 + ev] = {g.e, (R)0};
    }
    __syncthreads();
}
// gluon j's basis for this lane's event, re-read from LDS at every use (volatile, as lds_p4)
template <class R>
__device__ __forceinline__ GBT<R> lds_gb(const R* gbl, int j, int lane)
{
    typedef R v2 __attribute__((ext_vector_type(2)));
    typedef __attribute__((address_space(3))) const volatile v2 lds_v2;
    lds_v2* v = (lds_v2*)gbl;
    const v2 x = v[(3 * j) * 64 + lane], y = v[(3 * j + 1) * 64 + lane], z = v[(3 * j + 2) * 64 + lane];
    return {x.x, x.y, y.x, y.y, z.x};
}
template <class R>
__device__ __forceinline__ void pin_gb(GBT<R>& g)
{
    if constexpr (sizeof(R) == 8) asm volatile("" : "+v"(g.a), "+v"(g.b), "+v"(g.c), "+v"(g.d), "+v"(g.e));
}
// Marks a four-momentum as first needed here: arithmetic on it (momentum sums) cannot be
// moved above this point, so a value read from LDS early need not be waited for earlier.
// Only in the FP64 kernels (one wave per SIMD, nothing else hides the wait); the FP32
// kernels run two waves per SIMD and measured faster without it.
template <class R>
__device__ __forceinline__ void pin_p4(P4& p)
{
    if constexpr (sizeof(R) == 8) asm volatile("" : "+v"(p.t), "+v"(p.x), "+v"(p.y), "+v"(p.z));
}
// An external wavefunction kept in LDS, private to its lane, instead of in registers across
// the program: slot k holds component pairs (re, im) at xw[(4 k + m) * 64 + lane] (one 16-byte
// pair per lane in FP64, so a read is conflict-free).  ld_w4 re-reads it at every use
// (volatile, as lds_p4).
template <class R>
__device__ __forceinline__ void st_w4(R* xw, int k, int lane, const W4<R>& w)
{
    typedef R v2 __attribute__((ext_vector_type(2)));
    v2* p = reinterpret_cast<v2*>(xw);
#pragma unroll
    for (int m = 0; m < 4; ++m) p[(4 * k + m) * 64 + lane] = {w.c[m].r, w.c[m].i};
}
template <class R>
__device__ __forceinline__ W4<R> ld_w4(const R* xw, int k, int lane)
{
    typedef R v2 __attribute__((ext_vector_type(2)));
    typedef __attribute__((address_space(3))) const volatile v2 lds_v2;
    lds_v2* v = (lds_v2*)xw;
    W4<R> w;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const v2 t = v[(4 * k + m) * 64 + lane];
        w.c[m] = {t.x, t.y};
    }
    return w;
}
// as pin_p4, for an external wavefunction read ahead of the step that needs it
template <class R>
__device__ __forceinline__ void pin_w4(W4<R>& w)
{
    if constexpr (sizeof(R) == 8)
        asm volatile("" : "+v"(w.c[0].r), "+v"(w.c[0].i), "+v"(w.c[1].r), "+v"(w.c[1].i), "+v"(w.c[2].r),
                     "+v"(w.c[2].i), "+v"(w.c[3].r), "+v"(w.c[3].i));
}
// Makes an amplitude's value opaque once computed: the operations that produce it cannot be
// fused with those that consume it, so every instance of a kernel (with or without the
// channel-weight sums, whose extra uses of the value change what the compiler may contract)
// rounds it the same way.
template <class R>
__device__ __forceinline__ void pin_cx(cx<R>& a)
{
    asm volatile("" : "+v"(a.r), "+v"(a.i));
}
// LDS atomic add into this lane's private jamp slot (no return value: ds_add_f64 / ds_add_f32)
template <class R>
__device__ __forceinline__ void lds_add(R* p, R v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}
// jamp update in LDS: atomic add for double (ds_add_f64); plain read-add-write for float
// (the FP32 LDS atomic add is much slower than the FP64 one on gfx950).  A slot that
// receives atomic adds is also read and cleared with atomic accesses: plain loads and
// stores mixed with the no-return atomic adds on the same address were observed to be
// reordered in the compiled code, while accesses that are all atomic keep their order.
template <class R>
__device__ __forceinline__ void jamp_add(R* p, R v)
{
    if constexpr (sizeof(R) == 8) lds_add<R>(p, v);
    else *p += v;
}
template <class R>
__device__ __forceinline__ R jamp_get(R* p)
{
    if constexpr (sizeof(R) == 8) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    else return *p;
}
template <class R>
__device__ __forceinline__ void jamp_zero(R* p)
{
    if constexpr (sizeof(R) == 8) __hip_atomic_store(p, (R)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    else *p = (R)0;
}
}  // namespace me
