// fields.h -- field of one propagation path (Fresnel reflection with the
// polarisation tracked bounce by bounce, UTD edge diffraction), written once
// for a generic real type R:
//   R = double  the forward evaluation (k_fields),
//   R = DNT<N>  forward-mode dual numbers carrying derivatives with respect
//               to the transmitter position (3) and the dipole orientation
//               (theta, phi) (the adjoint, k_adj_paths).
// The permittivity derivatives use R = double with one interaction's
// reflection coefficients replaced by their derivatives (dmode).
//
// Field model (readings; the paper names reflection and diffraction in
// Section II-A, transmit power and an ideal omnidirectional antenna in
// Section IV, and fixes no formula):
//   specular: E = e_tx(k_0); at bounce i, with the face normal n turned
//   against the incident k_{i-1}: s = normalize(k_{i-1} x n) (normal
//   incidence: normalize(n x z), else normalize(n x x)), p_in = s x k_{i-1},
//   p_out = s x k_i, E <- Gamma_TE (E.s) s + Gamma_TM (E.p_in) p_out;
//   a = lambda / (4 pi L) (e_rx(k_K).E) exp(-j 2 pi frac(L / lambda)).
//   diffraction: a = lambda/(4 pi) (1/s') sqrt(s'/(s (s + s')))
//   e_rx.(D e_tx) exp(-j 2 pi frac((s + s')/lambda)), D = -b0 b0' D_s - ph ph' D_h,
//   Kouyoumjian-Pathak coefficients with Luebbers' lossy faces.
#pragma once
#include "emrt_dev.h"
#include "emrt_launch.h"

namespace emrt {

// ------------------------------------------------------- dual numbers ----
// DNT<N>: a value and its derivatives along N of the five tangent directions
// (d/d tx.x, tx.y, tx.z, theta, phi); DN carries all five, DN1 one of them.
constexpr int kTan = 5;
template <int N> struct DNT {
    double v;
    double d[N];
    static __device__ __forceinline__ DNT constant(double x) {
        DNT r;
        r.v = x;
#pragma unroll
        for (int k = 0; k < N; k++) r.d[k] = 0.0;
        return r;
    }
};
using DN = DNT<kTan>;
using DN1 = DNT<1>;
__device__ __forceinline__ DN dn(double v) { return DN::constant(v); }
// the value v of tangent direction k (0..4), carried by a number whose
// derivative slots hold directions first .. first + N - 1
template <int N> __device__ __forceinline__ DNT<N> dn_seed(double v, int k, int first = 0) {
    DNT<N> r = DNT<N>::constant(v);
#pragma unroll
    for (int j = 0; j < N; j++) r.d[j] = (first + j == k) ? 1.0 : 0.0;
    return r;
}
__device__ __forceinline__ DN dn_seed(double v, int k) { return dn_seed<kTan>(v, k, 0); }
template <int N> __device__ __forceinline__ DNT<N> operator+(DNT<N> a, DNT<N> b) {
    a.v += b.v;
#pragma unroll
    for (int k = 0; k < N; k++) a.d[k] += b.d[k];
    return a;
}
template <int N> __device__ __forceinline__ DNT<N> operator-(DNT<N> a, DNT<N> b) {
    a.v -= b.v;
#pragma unroll
    for (int k = 0; k < N; k++) a.d[k] -= b.d[k];
    return a;
}
template <int N> __device__ __forceinline__ DNT<N> operator-(DNT<N> a) {
    a.v = -a.v;
#pragma unroll
    for (int k = 0; k < N; k++) a.d[k] = -a.d[k];
    return a;
}
template <int N> __device__ __forceinline__ DNT<N> operator*(DNT<N> a, DNT<N> b) {
    DNT<N> r;
    r.v = a.v * b.v;
#pragma unroll
    for (int k = 0; k < N; k++) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
    return r;
}
template <int N> __device__ __forceinline__ DNT<N> operator/(DNT<N> a, DNT<N> b) {
    DNT<N> r;
    double inv = 1.0 / b.v;
    r.v = a.v * inv;
#pragma unroll
    for (int k = 0; k < N; k++) r.d[k] = (a.d[k] - r.v * b.d[k]) * inv;
    return r;
}
template <int N> __device__ __forceinline__ DNT<N> operator+(DNT<N> a, double b) { a.v += b; return a; }
template <int N> __device__ __forceinline__ DNT<N> operator+(double b, DNT<N> a) { a.v += b; return a; }
template <int N> __device__ __forceinline__ DNT<N> operator-(DNT<N> a, double b) { a.v -= b; return a; }
template <int N> __device__ __forceinline__ DNT<N> operator-(double b, DNT<N> a) { return DNT<N>::constant(b) - a; }
template <int N> __device__ __forceinline__ DNT<N> operator*(DNT<N> a, double s) {
    a.v *= s;
#pragma unroll
    for (int k = 0; k < N; k++) a.d[k] *= s;
    return a;
}
template <int N> __device__ __forceinline__ DNT<N> operator*(double s, DNT<N> a) { return a * s; }
template <int N> __device__ __forceinline__ DNT<N> operator/(DNT<N> a, double s) { return a * (1.0 / s); }
template <int N> __device__ __forceinline__ DNT<N> operator/(double s, DNT<N> b) { return DNT<N>::constant(s) / b; }

// scalar functions for both real types
__device__ __forceinline__ double vv(double x) { return x; }
template <int N> __device__ __forceinline__ double vv(const DNT<N>& x) { return x.v; }
__device__ __forceinline__ double sqrt_(double x) { return sqrt(x); }
template <int N> __device__ __forceinline__ DNT<N> sqrt_(DNT<N> a) {
    double s = sqrt(a.v);
    DNT<N> r = a * (0.5 / s);
    r.v = s;
    return r;
}
__device__ __forceinline__ double sin_(double x) { return sin(x); }
__device__ __forceinline__ double cos_(double x) { return cos(x); }
template <int N> __device__ __forceinline__ DNT<N> sin_(DNT<N> a) {
    double s, c;
    sincos(a.v, &s, &c);
    DNT<N> r = a * c;
    r.v = s;
    return r;
}
template <int N> __device__ __forceinline__ DNT<N> cos_(DNT<N> a) {
    double s, c;
    sincos(a.v, &s, &c);
    DNT<N> r = a * (-s);
    r.v = c;
    return r;
}
__device__ __forceinline__ double acos_(double x) { return acos(x); }
template <int N> __device__ __forceinline__ DNT<N> acos_(DNT<N> a) {
    DNT<N> r = a * (-1.0 / sqrt(1.0 - a.v * a.v));
    r.v = acos(a.v);
    return r;
}
__device__ __forceinline__ double atan2_(double y, double x) { return atan2(y, x); }
template <int N> __device__ __forceinline__ DNT<N> atan2_(DNT<N> y, DNT<N> x) {
    double inv = 1.0 / (x.v * x.v + y.v * y.v);
    DNT<N> r = (y * x.v - x * y.v) * inv;
    r.v = atan2(y.v, x.v);
    return r;
}
__device__ __forceinline__ double abs_(double x) { return fabs(x); }
template <int N> __device__ __forceinline__ DNT<N> abs_(DNT<N> a) { return a.v < 0 ? -a : a; }
template <class R> __device__ __forceinline__ R rl(double x) { return R::constant(x); }
template <> __device__ __forceinline__ double rl<double>(double x) { return x; }
template <class R> __device__ __forceinline__ R clamp1(R x) {
    if (vv(x) > 1.0) return rl<R>(1.0);
    if (vv(x) < -1.0) return rl<R>(-1.0);
    return x;
}

// ------------------------------------------------------------ vectors ----
template <class R> struct V3 { R x, y, z; };
template <class R> __device__ __forceinline__ V3<R> v3(R x, R y, R z) { return {x, y, z}; }
template <class R> __device__ __forceinline__ V3<R> v3c(dv3 a) { return {rl<R>(a.x), rl<R>(a.y), rl<R>(a.z)}; }
template <class R> __device__ __forceinline__ V3<R> operator+(V3<R> a, V3<R> b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class R> __device__ __forceinline__ V3<R> operator-(V3<R> a, V3<R> b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class R> __device__ __forceinline__ V3<R> operator+(V3<R> a, dv3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class R> __device__ __forceinline__ V3<R> operator-(V3<R> a, dv3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class R> __device__ __forceinline__ V3<R> operator-(dv3 a, V3<R> b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class R> __device__ __forceinline__ V3<R> operator*(V3<R> a, R s) { return {a.x * s, a.y * s, a.z * s}; }
template <class R> __device__ __forceinline__ V3<R> scale(V3<R> a, double s) { return {a.x * s, a.y * s, a.z * s}; }
template <class R> __device__ __forceinline__ V3<R> scale(dv3 a, R s) { return {s * a.x, s * a.y, s * a.z}; }
template <class R> __device__ __forceinline__ R dot3(V3<R> a, V3<R> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class R> __device__ __forceinline__ R dot3(dv3 a, V3<R> b) { return b.x * a.x + b.y * a.y + b.z * a.z; }
template <class R> __device__ __forceinline__ V3<R> cross3(V3<R> a, V3<R> b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <class R> __device__ __forceinline__ V3<R> cross3(dv3 a, V3<R> b) {
    return {b.z * a.y - b.y * a.z, b.x * a.z - b.z * a.x, b.y * a.x - b.x * a.y};
}
template <class R> __device__ __forceinline__ V3<R> cross3(V3<R> a, dv3 b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <class R> __device__ __forceinline__ R len3(V3<R> a) { return sqrt_(dot3(a, a)); }
template <class R> __device__ __forceinline__ V3<R> scale_inv(V3<R> a, R l) {
    R inv = 1.0 / l;
    return a * inv;
}
template <class R> __device__ __forceinline__ V3<R> unit3(V3<R> a) { return scale_inv(a, len3(a)); }
template <class R> __device__ __forceinline__ dv3 val3(V3<R> a) { return d3(vv(a.x), vv(a.y), vv(a.z)); }

// ------------------------------------------------------------ complex ----
template <class R> struct Cx { R re, im; };
template <class R> __device__ __forceinline__ Cx<R> cx(R re, R im) { return {re, im}; }
template <class R> __device__ __forceinline__ Cx<R> cxc(cd a) { return {rl<R>(a.re), rl<R>(a.im)}; }
template <class R> __device__ __forceinline__ Cx<R> operator+(Cx<R> a, Cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <class R> __device__ __forceinline__ Cx<R> operator-(Cx<R> a, Cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <class R> __device__ __forceinline__ Cx<R> operator*(Cx<R> a, Cx<R> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class R> __device__ __forceinline__ Cx<R> operator*(Cx<R> a, R s) { return {a.re * s, a.im * s}; }
template <class R> __device__ __forceinline__ Cx<R> cmul(Cx<R> a, cd b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class R> __device__ __forceinline__ Cx<R> cscale(Cx<R> a, double s) { return {a.re * s, a.im * s}; }
template <class R> __device__ __forceinline__ Cx<R> cdivx(Cx<R> a, Cx<R> b) {
    R den = b.re * b.re + b.im * b.im;
    R inv = 1.0 / den;
    return {(a.re * b.re + a.im * b.im) * inv, (a.im * b.re - a.re * b.im) * inv};
}
// double: Smith's division (as the forward path has always used)
template <> __device__ __forceinline__ Cx<double> cdivx<double>(Cx<double> a, Cx<double> b) {
    cd r = cdiv(C(a.re, a.im), C(b.re, b.im));
    return {r.re, r.im};
}
template <int N> __device__ __forceinline__ Cx<DNT<N>> csqrt_dual(Cx<DNT<N>> z) {
    // w = sqrt(z): dw = dz / (2 w)
    cd w = csqrtd(C(z.re.v, z.im.v));
    cd h = cdiv(C(0.5), w);
    Cx<DNT<N>> r;
    r.re.v = w.re;
    r.im.v = w.im;
#pragma unroll
    for (int k = 0; k < N; k++) {
        r.re.d[k] = z.re.d[k] * h.re - z.im.d[k] * h.im;
        r.im.d[k] = z.re.d[k] * h.im + z.im.d[k] * h.re;
    }
    return r;
}
template <class R> __device__ __forceinline__ Cx<R> csqrtx(Cx<R> z) { return csqrt_dual(z); }
template <> __device__ __forceinline__ Cx<double> csqrtx<double>(Cx<double> z) {
    cd r = csqrtd(C(z.re, z.im));
    return {r.re, r.im};
}
template <class R> __device__ __forceinline__ Cx<R> cdotx(V3<R> a, const Cx<R>* E) {
    return {a.x * E[0].re + a.y * E[1].re + a.z * E[2].re, a.x * E[0].im + a.y * E[1].im + a.z * E[2].im};
}

// --------------------------------------------------------- ingredients ----
// Fresnel coefficients of a half space of relative permittivity eps
// (eps' - j eps'', time factor exp(+j w t)) at incidence cosine c, principal
// square root r = sqrt(eps - sin^2):
//   Gamma_TE = (c - r) / (c + r),  Gamma_TM = (eps c - r) / (eps c + r);
// with deriv set, their derivatives with respect to eps:
//   dGamma_TE = -c / (r (c + r)^2),  dGamma_TM = c (eps - 2 sin^2) / (r (eps c + r)^2).
template <class R>
__device__ __forceinline__ void fresnel_x(cd eps, R c, bool deriv, Cx<R>& te, Cx<R>& tm) {
    R s2 = 1.0 - c * c;
    Cx<R> z = cx<R>(eps.re - s2, rl<R>(eps.im));
    Cx<R> r = csqrtx(z);
    Cx<R> cc = cx<R>(c, rl<R>(0.0));
    Cx<R> ec = cx<R>(c * eps.re, c * eps.im);
    if (!deriv) {
        te = cdivx(cc - r, cc + r);
        tm = cdivx(ec - r, ec + r);
        return;
    }
    Cx<R> cr = cc + r, er = ec + r;
    te = cdivx(cx<R>(-c, rl<R>(0.0)), r * cr * cr);
    Cx<R> num = cx<R>(c * (eps.re - 2.0 * s2), c * eps.im);
    tm = cdivx(num, r * er * er);
}

// Reflection coefficients of material m.  Table I (Section IV) gives its
// surfaces a reflection coefficient alone; where fc.mat_refl[m] = g > 0 the
// coefficient is that magnitude at every angle and for both polarisations,
// with a perfect conductor's signs in this basis (the eps -> infinity limit of
// fresnel_x: TE -g, TM +g), and has no permittivity derivative.  Otherwise
// the Fresnel coefficients of the material's permittivity.
template <class R>
__device__ __forceinline__ void material_x(const FieldCtx& fc, int m, R c, bool deriv, Cx<R>& te, Cx<R>& tm) {
    const double g = fc.mat_refl[m];
    if (g > 0.0) {
        const double s = deriv ? 0.0 : g;
        te = cx<R>(rl<R>(-s), rl<R>(0.0));
        tm = cx<R>(rl<R>(s), rl<R>(0.0));
        return;
    }
    fresnel_x<R>(C(fc.mat_eps[2 * m], fc.mat_eps[2 * m + 1]), c, deriv, te, tm);
}

// erfcx(w) = exp(w^2) erfc(w) on w = exp(j pi/4) v, v >= 0: power series of
// erf for v < 2.5 (Abramowitz & Stegun 7.1.5), Laplace continued fraction
// (A&S 7.1.14) by the modified Lentz method otherwise.  Moduli are compared
// squared, and the reciprocals of the Lentz recurrences are conj(z) / |z|^2
// with one real division for both (|z| stays between about 1 and 1e3 here,
// far from overflow or underflow).
__device__ inline cd erfcx_diag(double v) {
    const double h = 0.70710678118654752440;
    cd w = C(v * h, v * h);
    if (v < 2.5) {
        cd w2 = w * w;
        cd term = w, sum = w;
        for (int n = 1; n < 400; n++) {
            term = term * (w2 * (-1.0 / (double)n));
            cd add = term * (1.0 / (double)(2 * n + 1));
            sum = sum + add;
            if (cabs2(add) < 1e-36 * cabs2(sum) + 1e-300) break;
        }
        cd erfc_w = C(1.0) - sum * (2.0 / sqrt(kPi));
        return cexpi(v * v) * erfc_w;  // exp(w^2), w^2 = j v^2
    }
    const double tiny = 1e-300;
    cd f = w, Cc = w, D = C(0.0);
    for (int n = 1; n < 5000; n++) {
        double an = 0.5 * n;
        D = w + D * an;
        if (fmax(fabs(D.re), fabs(D.im)) < tiny) D = C(tiny);
        // Cc = w + an / Cc and D = 1 / D, both through one division
        const double nc = cabs2(Cc), nd = cabs2(D);
        const double r = 1.0 / (nc * nd);
        const double sc = an * nd * r, sd = nc * r;  // an / |Cc|^2, 1 / |D|^2
        Cc = C(w.re + Cc.re * sc, w.im - Cc.im * sc);
        if (fmax(fabs(Cc.re), fabs(Cc.im)) < tiny) Cc = C(tiny);
        D = C(D.re * sd, -D.im * sd);
        cd delta = Cc * D;
        f = f * delta;
        // a few ulps of 1: the rounded product of converged factors can sit
        // one ulp below 1 for good, so a tighter test may never be met
        if (cabs2(delta - C(1.0)) < 1e-30) break;
    }
    return cdiv(C(1.0), f * sqrt(kPi));
}

// UTD transition function F(X) = e^{j pi/4} sqrt(pi X) erfcx(e^{j pi/4} sqrt X)
// (Kouyoumjian & Pathak 1974), X >= 0; F'(X) = F (j + 1/(2X)) - j.
__device__ inline cd utd_F(double X) {
    if (X <= 0) return C(0.0);
    const double h = 0.70710678118654752440;
    return C(h, h) * erfcx_diag(sqrt(X)) * sqrt(kPi * X);
}
template <int N> __device__ __forceinline__ Cx<DNT<N>> utd_F_dual(DNT<N> X) {
    cd f = utd_F(X.v);
    cd df = X.v > 0 ? f * C(0.5 / X.v, 1.0) - C(0.0, 1.0) : C(0.0);
    Cx<DNT<N>> r;
    r.re.v = f.re;
    r.im.v = f.im;
#pragma unroll
    for (int k = 0; k < N; k++) {
        r.re.d[k] = df.re * X.d[k];
        r.im.d[k] = df.im * X.d[k];
    }
    return r;
}
template <class R> __device__ __forceinline__ Cx<R> utd_Fx(R X) { return utd_F_dual(X); }
template <> __device__ __forceinline__ Cx<double> utd_Fx<double>(double X) {
    cd f = utd_F(X);
    return {f.re, f.im};
}

// cot((pi + sg beta)/(2n)) F(kL a^{sg}(beta)), a = 2 cos^2((2 pi n N - beta)/2),
// N the integer nearest (beta + sg pi)/(2 pi n); within |eps| < 1e-4 of a
// shadow or reflection boundary (eps = pi + sg (beta - 2 pi n N)) the finite
// limit n e^{j pi/4} [sqrt(2 pi kL) sgn(eps) - 2 kL eps e^{j pi/4}].
template <class R>
__device__ __forceinline__ Cx<R> utd_term_x(double sg, R beta, double n, R kL) {
    double N = rint((vv(beta) + sg * kPi) / (2.0 * kPi * n));
    R eps = kPi + sg * (beta - 2.0 * kPi * n * N);
    const double h = 0.70710678118654752440;
    if (fabs(vv(eps)) < 1e-4) {
        double sgn = vv(eps) > 0 ? 1.0 : (vv(eps) < 0 ? -1.0 : 0.0);
        // e4 (sqrt(2 pi kL) sgn - e4 2 kL eps) n, e4 = (h, h), e4^2 = j
        R a = sqrt_(2.0 * kPi * kL) * (sgn * n);
        R b = kL * eps * (2.0 * n);
        // e4 * a - j * b
        return cx<R>(a * h, a * h - b);
    }
    R c = cos_((2.0 * kPi * n * N - beta) * 0.5);
    R x = (kPi + sg * beta) / (2.0 * n);
    R cot = cos_(x) / sin_(x);
    return utd_Fx<R>(kL * 2.0 * c * c) * cot;
}

// Kouyoumjian-Pathak coefficient with Luebbers' lossy-face factors: R_0 of
// the 0-face at incidence cosine sin(beta0)|sin phi'|, R_n of the n-face at
// sin(beta0)|sin(n pi - phi)|, TE for soft and TM for hard:
//   D = Cc [T(+, phi - phi') + T(-, phi - phi') + R_n T(+, phi + phi') + R_0 T(-, phi + phi')],
//   Cc = -e^{-j pi/4} / (2 n sqrt(2 pi k) sin beta0).
// R_0 and R_n are the coefficients of the faces' materials m0 and mn
// (material_x).  dmode 1 / 2: the derivative with respect to the 0-face /
// n-face permittivity.
template <class R>
__device__ __forceinline__ void utd_D_x(double n, double k, R L, R beta0, R php, R ph, const FieldCtx& fc, int m0,
                                        int mn, int dmode, Cx<R>& Ds, Cx<R>& Dh) {
    R sb = sin_(beta0);
    const double h = 0.70710678118654752440;
    R cmag = 1.0 / ((2.0 * n * sqrt(2.0 * kPi * k)) * sb);
    Cx<R> Cc = cx<R>(cmag * (-h), cmag * h);
    R kL = L * k;
    // the four terms one at a time (one transition function live, not four):
    // k = 0, 1 the incident-shadow pair (ph - php, summed), 2, 3 the
    // reflection-shadow terms (ph + php); derivative modes need only one
    Cx<R> t12 = cx<R>(rl<R>(0.0), rl<R>(0.0)), t3 = t12, t4 = t12;
#pragma unroll 1
    for (int j = 0; j < 4; j++) {
        if ((dmode == 1 && j != 3) || (dmode == 2 && j != 2)) continue;
        const Cx<R> t = utd_term_x<R>((j & 1) ? -1 : +1, j < 2 ? ph - php : ph + php, n, kL);
        if (j < 2) t12 = t12 + t;
        else if (j == 2) t3 = t;
        else t4 = t;
    }
    Cx<R> r0te, r0tm, rnte, rntm;
    material_x<R>(fc, m0, sb * abs_(sin_(php)), dmode == 1, r0te, r0tm);
    material_x<R>(fc, mn, sb * abs_(sin_(n * kPi - ph)), dmode == 2, rnte, rntm);
    if (dmode == 0) {
        Ds = Cc * (t12 + rnte * t3 + r0te * t4);
        Dh = Cc * (t12 + rntm * t3 + r0tm * t4);
    } else if (dmode == 1) {
        Ds = Cc * (r0te * t4);
        Dh = Cc * (r0tm * t4);
    } else {
        Ds = Cc * (rnte * t3);
        Dh = Cc * (rntm * t3);
    }
}

// transmit / receive polarisation: vertical iso (mode 0; x when k is along z)
// or a short dipole along u(theta, phi) (mode 1): e = sqrt(1.5) (u - (u.k) k)
template <class R>
__device__ __forceinline__ V3<R> antenna_x(int mode, V3<R> k, R th, R ph) {
    if (mode == 1) {
        R st = sin_(th), ct = cos_(th), sp = sin_(ph), cp = cos_(ph);
        V3<R> u = v3<R>(st * cp, st * sp, ct);
        V3<R> e = u - k * dot3(u, k);
        return scale(e, sqrt(1.5));
    }
    V3<R> e = v3<R>(rl<R>(0.0) - k.x * k.z, rl<R>(0.0) - k.y * k.z, 1.0 - k.z * k.z);
    if (sqrt(vv(dot3(e, e))) < 1e-12) e = v3<R>(1.0 - k.x * k.x, rl<R>(0.0) - k.y * k.x, rl<R>(0.0) - k.z * k.x);
    return unit3(e);
}

// exp(-j 2 pi frac(L / lambda)) (frac taken on the value; derivative -j k dL)
template <int N> __device__ __forceinline__ Cx<DNT<N>> phase_dual(DNT<N> L, double lam) {
    double x = L.v / lam;
    cd p = cexpi(-2.0 * kPi * (x - rint(x)));
    double kk = 2.0 * kPi / lam;
    Cx<DNT<N>> r;
    r.re.v = p.re;
    r.im.v = p.im;
    // d p = -j k p dL
#pragma unroll
    for (int k = 0; k < N; k++) {
        r.re.d[k] = kk * p.im * L.d[k];
        r.im.d[k] = -kk * p.re * L.d[k];
    }
    return r;
}
template <class R> __device__ __forceinline__ Cx<R> phase_x(R L, double lam) { return phase_dual(L, lam); }
template <> __device__ __forceinline__ Cx<double> phase_x<double>(double L, double lam) {
    double x = L / lam;
    cd p = cexpi(-2.0 * kPi * (x - rint(x)));
    return {p.re, p.im};
}

// ------------------------------------------------------ wedge geometry ----
struct Wedge {
    dv3 P0, e, t0, n0;
    double len, n;
    int f0, fn;
};

__device__ __forceinline__ dv3 vert(const SceneDev& s, int v) { return ldf3(s.verts + 3 * (long long)v); }

__device__ __forceinline__ Wedge wedge_of(const SceneDev& s, int e) {
#pragma clang fp contract(off)
    const int* row = s.edge_i + 6 * (long long)e;
    Wedge w;
    w.P0 = vert(s, row[0]);
    dv3 ev = vert(s, row[1]) - w.P0;
    w.len = len(ev);
    w.e = ev * (1.0 / w.len);
    dv3 r0 = vert(s, row[4]) - w.P0, rn = vert(s, row[5]) - w.P0;
    w.t0 = unit(r0 - w.e * dot(r0, w.e));
    dv3 tn = unit(rn - w.e * dot(rn, w.e));
    dv3 n0 = cross(w.e, w.t0);
    if (dot(n0, tn) > 0) n0 = n0 * -1.0;
    w.n0 = n0;
    w.n = s.edge_n[e];
    w.f0 = row[2];
    w.fn = row[3];
    return w;
}

// angle of p about the edge, measured from the 0-face into the exterior, [0, 2 pi)
__device__ __forceinline__ double wedge_angle(const Wedge& w, dv3 p) {
#pragma clang fp contract(off)
    dv3 v = p - w.P0;
    double ph = atan2(dot(v, w.n0), dot(v, w.t0));
    if (ph < 0) ph += 2.0 * kPi;
    return ph;
}
template <class R>
__device__ __forceinline__ R wedge_angle_x(const Wedge& w, V3<R> p) {
    V3<R> v = p - w.P0;
    R ph = atan2_(dot3(w.n0, v), dot3(w.t0, v));
    if (vv(ph) < 0) ph = ph + 2.0 * kPi;
    return ph;
}

// ------------------------------------------------------ path geometry ----
// Points of a path: P[0] = Tx, P[1..order] reflection points (or P[1] = the
// Keller point), Rx last; np = points including both ends.
template <class R>
struct PathGeo {
    V3<R> P[EMRT_KMAX + 2];
    V3<R> Rx;
    int np, order, type;
};

// Interaction points of a key with its topology held fixed (no range,
// containment or occlusion test): image method for reflections, closed-form
// Keller point for diffraction.  Used by the adjoint, where the derivatives
// of the points with respect to the transmitter flow through R.
// KIND (as for path_field): 0 any type, 1 line of sight / specular only,
// 2 diffraction alone only, 3 one reflection and one diffraction only,
// 4 any type but the last.
template <class R, int KIND = 0>
__device__ __forceinline__ void path_points(const SceneDev& S, const KeyRec& key, V3<R> s, dv3 rx, PathGeo<R>& g) {
#pragma clang fp contract(off)
    g.type = key.to & 0xff;
    g.order = key.to >> 8;
    g.P[0] = s;
    g.Rx = v3c<R>(rx);
    if (g.type == KT_LOS) {
        g.np = 2;
        return;
    }
    // KIND 2 and 3 take only their own type: the branches below it are not compiled in
    if (KIND == 2 || ((KIND == 0 || KIND == 4) && g.type == KT_DIFF)) {
        g.np = 3;
        Wedge w = wedge_of(S, key.ids[0]);
        R zs = dot3(w.e, s - w.P0);
        double zr = dot(w.e, rx - w.P0);
        R rs = len3((s - w.P0) - scale(w.e, zs));
        dv3 rr3 = rx - w.P0 - w.e * zr;
        double rr = len(rr3);
        R zq = zs + (zr - zs) * rs / (rs + rr);
        g.P[1] = scale(w.e, zq) + w.P0;
        return;
    }
    if (KIND == 3 || (KIND == 0 && (g.type == KT_RD || g.type == KT_DR))) {
        // the Keller point between the unfolded ends (Tx's image and Rx, or Tx
        // and Rx's image), then the reflection point on the segment from it to
        // the image
        const bool rd = g.type == KT_RD;
        g.np = 4;
        Wedge w = wedge_of(S, rd ? key.ids[1] : key.ids[0]);
        const double* pl = S.plane + 4 * (long long)(rd ? key.ids[0] : key.ids[1]);
        dv3 n = d3(pl[0], pl[1], pl[2]);
        V3<R> a = s, b = g.Rx;
        if (rd) a = s - scale(n, (dot3(n, s) - pl[3]) * 2.0);
        else b = g.Rx - scale(n, (dot3(n, g.Rx) - pl[3]) * 2.0);
        R za = dot3(w.e, a - w.P0), zb = dot3(w.e, b - w.P0);
        R ra = len3((a - w.P0) - scale(w.e, za)), rb = len3((b - w.P0) - scale(w.e, zb));
        R zq = za + (zb - za) * ra / (ra + rb);
        V3<R> Q = scale(w.e, zq) + w.P0;
        V3<R> dv = (rd ? a : b) - Q;
        R tt = (pl[3] - dot3(n, Q)) / dot3(n, dv);
        V3<R> P = Q + dv * tt;
        g.P[1] = rd ? P : Q;
        g.P[2] = rd ? Q : P;
        return;
    }
    const int order = g.order;
    g.np = order + 2;
    V3<R> img[EMRT_KMAX + 1];
    img[0] = s;
#pragma unroll
    for (int i = 1; i <= EMRT_KMAX; i++) {
        if (i > order) break;
        const double* pl = S.plane + 4 * (long long)key.ids[i - 1];
        dv3 n = d3(pl[0], pl[1], pl[2]);
        R t = (dot3(n, img[i - 1]) - pl[3]) * 2.0;
        img[i] = img[i - 1] - scale(n, t);
    }
    V3<R> cur = g.Rx;
#pragma unroll
    for (int i = EMRT_KMAX; i >= 1; i--) {
        if (i > order) continue;
        const double* pl = S.plane + 4 * (long long)key.ids[i - 1];
        dv3 n = d3(pl[0], pl[1], pl[2]);
        V3<R> dv = img[i] - cur;
        R tt = (pl[3] - dot3(n, cur)) / dot3(n, dv);
        cur = cur + dv * tt;
        g.P[i] = cur;
    }
}

// Leg directions k_i, the unfolded length L and the complex amplitude of
// every carrier.  dmode = 0: the field; dmode = i >= 1 (specular): the
// derivative with respect to the permittivity of bounce i's material;
// dmode = 1 / 2 (diffraction): with respect to the 0-face / n-face material,
// 3 (one reflection with one diffraction): the reflection face's.
// KIND = 1 / 2 / 3 compiles only the line-of-sight-and-specular / the
// diffraction-alone / the combined paths (the caller guarantees the path
// type); 4 all but the combined paths; 0 everything.
// Reflection of the complex field vector E travelling along ki into ko at
// face f, in the bounce's s/p basis (s = normalize(ki x n), n against ki;
// normal incidence: n x z, else n x x): E <- Gamma_TE (E.s) s +
// Gamma_TM (E.p_in) p_out, with p = s x k; deriv: the coefficients'
// permittivity derivatives instead.
template <class R>
__device__ __forceinline__ void reflect_x(const SceneDev& S, const FieldCtx& fc, int f, V3<R> ki, V3<R> ko, bool deriv,
                                          Cx<R>* E) {
    const double* pl = S.plane + 4 * (long long)f;
    dv3 nrm = d3(pl[0], pl[1], pl[2]);
    if (vv(dot3(nrm, ki)) > 0) nrm = nrm * -1.0;
    R c = rl<R>(0.0) - dot3(nrm, ki);
    V3<R> sv = cross3(ki, nrm);
    if (sqrt(vv(dot3(sv, sv))) < 1e-12) {
        sv = v3c<R>(cross(nrm, d3(0, 0, 1)));
        if (sqrt(vv(dot3(sv, sv))) < 1e-12) sv = v3c<R>(cross(nrm, d3(1, 0, 0)));
    }
    sv = unit3(sv);
    V3<R> pin = cross3(sv, ki), pout = cross3(sv, ko);
    Cx<R> te, tm;
    material_x<R>(fc, S.face_material[f], c, deriv, te, tm);
    Cx<R> es = cdotx(sv, E) * te, ep = cdotx(pin, E) * tm;
    E[0] = es * sv.x + ep * pout.x;
    E[1] = es * sv.y + ep * pout.y;
    E[2] = es * sv.z + ep * pout.z;
}

template <class R, int KIND = 0>
__device__ __forceinline__ void path_field(const SceneDev& S, const FieldCtx& fc, const KeyRec& key, const PathGeo<R>& g,
                                           R th, R phi, int dmode, V3<R>* kk, R& L, Cx<R>* amp) {
    L = rl<R>(0.0);
    // legs of a path of this kind at most (diffraction alone: 2, with one reflection: 3)
    constexpr int kLegs = KIND == 2 ? 2 : (KIND == 3 ? 3 : EMRT_KMAX + 1);
#pragma unroll
    for (int i = 0; i < kLegs; i++) {
        if (i + 1 >= g.np) break;
        V3<R> p1 = (i + 2 == g.np) ? g.Rx : g.P[i + 1 <= EMRT_KMAX + 1 ? i + 1 : EMRT_KMAX + 1];
        V3<R> dv = p1 - g.P[i];
        R l = len3(dv);
        L = L + l;
        kk[i] = scale_inv(dv, l);
    }
    const int nlegs = g.np - 1;
    V3<R> k0 = kk[0];
    V3<R> kK = kk[0];
#pragma unroll
    for (int i = 1; i < kLegs; i++)
        if (i == nlegs - 1) kK = kk[i];
    const bool diffracted = (KIND == 2 || KIND == 3) ? true : (KIND == 1 ? false : g.type >= KT_DIFF);
    if (!diffracted) {
        V3<R> e0 = antenna_x<R>(fc.ant_mode, k0, th, phi);
        V3<R> er = antenna_x<R>(0, kK, rl<R>(0.0), rl<R>(0.0));
        for (int fi = 0; fi < fc.nf; fi++) {
            double lam = kC0 / fc.freq[fi];
            Cx<R> E[3] = {cx<R>(e0.x, rl<R>(0.0)), cx<R>(e0.y, rl<R>(0.0)), cx<R>(e0.z, rl<R>(0.0))};
#pragma unroll
            for (int i = 1; i <= EMRT_KMAX; i++) {
                if (i > g.order || g.type == KT_LOS) break;
                reflect_x<R>(S, fc, key.ids[i - 1], kk[i - 1], kk[i], dmode == i, E);
            }
            R scl = lam / (4.0 * kPi * L);
            amp[fi] = cdotx(er, E) * phase_x<R>(L, lam) * scl;
        }
    } else {
        // diffraction alone, or after (RD) / before (DR) one reflection: points
        // Tx, [P], Q, [P], Rx; sp / sd are the unfolded lengths on the source /
        // receiver side of the Keller point Q; the reflection acts on the field
        // vector arriving at Q (RD) or leaving it (DR).  dmode 1 / 2: the wedge
        // faces' permittivity derivative, 3: the reflection face's.
        // KIND 2 and 4 leave the combined paths out, KIND 3 the diffraction alone
        const bool comb = KIND == 0 || KIND == 3;
        const bool rd = comb && g.type == KT_RD, dr = comb && g.type == KT_DR;
        Wedge w = wedge_of(S, rd ? key.ids[1] : key.ids[0]);
        const int iq = rd ? 1 : 0;  // leg arriving at Q
        V3<R> si = kk[iq], so = kk[iq + 1];
        R sp, sd;
        if (rd) {
            sp = len3(g.P[1] - g.P[0]) + len3(g.P[2] - g.P[1]);
            sd = len3(g.Rx - g.P[2]);
        } else if (dr) {
            sp = len3(g.P[1] - g.P[0]);
            sd = len3(g.P[2] - g.P[1]) + len3(g.Rx - g.P[2]);
        } else {
            sp = len3(g.P[1] - g.P[0]);
            sd = len3(g.Rx - g.P[1]);
        }
        R cb = clamp1<R>(dot3(si, v3c<R>(w.e)));
        R beta0 = acos_(cb);
        R php = wedge_angle_x<R>(w, rd ? g.P[1] : g.P[0]), ph = wedge_angle_x<R>(w, dr ? g.P[2] : g.Rx);
        R sb = sin_(beta0);
        R Lp = sd * sp * sb * sb / (sd + sp);
        V3<R> fp = scale(unit3(cross3(w.e, si)), -1.0), bp = cross3(fp, si);
        V3<R> fo = unit3(cross3(w.e, so)), bo = cross3(fo, so);
        int m0 = S.face_material[w.f0], mn = S.face_material[w.fn];
        V3<R> et = antenna_x<R>(fc.ant_mode, k0, th, phi);
        V3<R> er = antenna_x<R>(0, kK, rl<R>(0.0), rl<R>(0.0));
        R spread = (1.0 / sp) * sqrt_(sp / (sd * (sd + sp)));
        const int wmode = dmode == 3 ? 0 : dmode;
        if (KIND != 3 && !rd && !dr) {
            R cs = rl<R>(0.0) - dot3(er, bo) * dot3(bp, et);
            R ch = dot3(er, fo) * dot3(fp, et);
            // KIND 2 is called one carrier at a time (the field kernel splits the carriers)
            const int nf = KIND == 2 ? 1 : fc.nf;
            for (int fi = 0; fi < nf; fi++) {
                double lam = kC0 / fc.freq[fi];
                double k = 2.0 * kPi / lam;
                Cx<R> Ds, Dh;
                utd_D_x<R>(w.n, k, Lp, beta0, php, ph, fc, m0, mn, wmode, Ds, Dh);
                Cx<R> fld = Ds * cs - Dh * ch;
                amp[fi] = fld * phase_x<R>(L, lam) * (spread * (lam / (4.0 * kPi)));
            }
        } else {
            const int fr = rd ? key.ids[0] : key.ids[1];
            for (int fi = 0; fi < fc.nf; fi++) {
                double lam = kC0 / fc.freq[fi];
                double k = 2.0 * kPi / lam;
                Cx<R> Ds, Dh;
                utd_D_x<R>(w.n, k, Lp, beta0, php, ph, fc, m0, mn, wmode, Ds, Dh);
                Cx<R> E[3] = {cx<R>(et.x, rl<R>(0.0)), cx<R>(et.y, rl<R>(0.0)), cx<R>(et.z, rl<R>(0.0))};
                if (rd) reflect_x<R>(S, fc, fr, kk[0], kk[1], dmode == 3, E);
                // diffracted field vector: -b0 (b0'.E) D_s - phi (phi'.E) D_h
                Cx<R> cbs = cdotx(bp, E) * Ds, cfh = cdotx(fp, E) * Dh;
                Cx<R> Ed[3] = {cx<R>(rl<R>(0.0), rl<R>(0.0)) - cbs * bo.x - cfh * fo.x,
                               cx<R>(rl<R>(0.0), rl<R>(0.0)) - cbs * bo.y - cfh * fo.y,
                               cx<R>(rl<R>(0.0), rl<R>(0.0)) - cbs * bo.z - cfh * fo.z};
                if (dr) reflect_x<R>(S, fc, fr, kk[1], kk[2], dmode == 3, Ed);
                amp[fi] = cdotx(er, Ed) * phase_x<R>(L, lam) * (spread * (lam / (4.0 * kPi)));
            }
        }
    }
}

}  // namespace emrt
