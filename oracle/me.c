/* oracle/me.c -- plain, slow CPU reference for the leading-order |M|^2.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the bench's cpu_baseline
 * leg may load or call it; the product path never does.  It shares no code, header,
 * table or generator with the HIP library.  The file is compiled twice: with
 * OR_REAL=double (liboracle.so) and with OR_REAL=long double (liboracle_ld.so, the
 * referee for ill-conditioned events).
 *
 * What it computes.  The paper's hot path is the per-event matrix element of a tree-level
 * process, computed independently for every phase-space event (Sec. 1) for the process
 * set of Sec. 2 (e+e- -> mu+mu-, gg -> tt~ with 0..3 extra gluons).  The paper prints no
 * formula; the quantity is the textbook one:
 *
 *     ME(p) = 1/A * sum_{helicities} sum_{colours} |M(p)|^2
 *
 * with M the sum of all tree-level Feynman diagrams in Feynman gauge, A the number of
 * initial spin x colour states (4 for e+e-, 4*64 for gg), final states summed, and no
 * identical-particle factor.  Conventions: metric (+,-,-,-); momenta (E,px,py,pz) in GeV;
 * Dirac matrices in the chiral representation; Feynman rules of Peskin & Schroeder
 * ch. 16 (quark-gluon vertex i g gamma^mu t^a, three-gluon vertex g f^{abc}[...],
 * four-gluon vertex -i g^2 [f f (..) + ..], propagators i(pslash+m)/(p^2-m^2) and
 * -i g_{mu nu}/p^2), t^a = lambda^a/2 with the Gell-Mann matrices.
 *
 * How.  Not the Feynman-diagram program the GPU runs, but:
 *   - QCD: colour decomposition M = sum_sigma (t^{a_sigma1}..t^{a_sigman})_{i j} A(sigma)
 *     (one quark line, Mangano & Parke, Phys. Rep. 200 (1991) 301), with the colour-
 *     ordered A(sigma) from the Berends-Giele recursion (Nucl. Phys. B306 (1988) 759) and
 *     the colour matrix C = sum over explicit colour indices of (T^sigma)(T^tau)^*,
 *     summed numerically with the Gell-Mann matrices;
 *   - gg -> gg (a test process): the single-trace decomposition with leg 4 fixed last;
 *   - e+e- -> mu+mu-: the one photon diagram written out as a spinor sandwich, and with Z
 *     exchange added (chiral couplings, Breit-Wigner propagator);
 *   - a colour-dressed recursion with explicit f^{abc} and t^a and explicit external
 *     colours, used to brute-force the colour sum and to spot-check the decomposition;
 *   - one Feynman diagram at a time (or_tree_amp, colour stripped): the single-diagram
 *     channel weights and the FP64 conditioning of a diagram sum are built on it in
 *     oracle/diagrams.py, with its own diagram enumeration and numeric colour factors.
 * External states are helicity eigenstates (the HELAS conventions: Hagiwara, Murayama,
 * Watanabe, KEK-91-11), plus a second basis (linear gluon polarisations, top spin along z
 * in the rest frame) for basis-independence checks.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <tgmath.h>

#ifndef OR_REAL
#define OR_REAL double
#endif
typedef OR_REAL real;
typedef OR_REAL _Complex cplx;

#define PI_R ((real)3.141592653589793238462643383279502884L)
#define NG_MAX 5
#define NPERM_MAX 120

enum { P_EE_MUMU = 0, P_GG_TT = 1, P_GG_TTG = 2, P_GG_TTGG = 3, P_GG_TTGGG = 4, P_GG_GG = 5,
       P_EE_MUMU_Z = 6, N_PROC = 7 };
static const int N_PAR[N_PROC] = {4, 4, 5, 6, 7, 4, 4};
static int is_qcd(int proc) { return proc >= P_GG_TT && proc <= P_GG_GG; }
static int is_ee(int proc) { return proc == P_EE_MUMU || proc == P_EE_MUMU_Z; }
/* electroweak constants of ee -> mumu with Z exchange: M_Z, Gamma_Z [GeV], M_W [GeV]
 * (sin^2 theta_W = 1 - M_W^2 / M_Z^2) */
#define EW_MZ ((real)91.188L)
#define EW_WZ ((real)2.441404L)
#define EW_MW ((real)80.419L)

/* ------------------------------------------------------------------------------------ */
/* constant tables: Dirac matrices, SU(3) generators, structure constants                */

static cplx GAM[4][4][4];         /* gamma^mu, chiral representation                    */
static cplx TA[8][3][3];          /* t^a = lambda^a / 2                                  */
static real FABC[8][8][8];        /* f^{abc} = -2 i Tr([t^a, t^b] t^c)                    */
static real FF[3][8][8][8][8];    /* sum_e f^{abe}f^{cde}, f^{ace}f^{bde}, f^{ade}f^{bce} */
static pthread_once_t tables_once = PTHREAD_ONCE_INIT;

static void init_tables(void)
{
    /* sigma^mu = (1, sigma_x, sigma_y, sigma_z); sigmabar^mu = (1, -sigma_k) */
    cplx s[4][2][2] = {
        {{1, 0}, {0, 1}},
        {{0, 1}, {1, 0}},
        {{0, -I}, {I, 0}},
        {{1, 0}, {0, -1}},
    };
    memset(GAM, 0, sizeof GAM);
    for (int mu = 0; mu < 4; ++mu)
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) {
                GAM[mu][i][j + 2] = s[mu][i][j];                        /* sigma^mu    */
                GAM[mu][i + 2][j] = (mu == 0) ? s[0][i][j] : -s[mu][i][j]; /* sigmabar^mu */
            }

    /* Gell-Mann matrices */
    cplx lam[8][3][3];
    memset(lam, 0, sizeof lam);
    lam[0][0][1] = 1;  lam[0][1][0] = 1;
    lam[1][0][1] = -I; lam[1][1][0] = I;
    lam[2][0][0] = 1;  lam[2][1][1] = -1;
    lam[3][0][2] = 1;  lam[3][2][0] = 1;
    lam[4][0][2] = -I; lam[4][2][0] = I;
    lam[5][1][2] = 1;  lam[5][2][1] = 1;
    lam[6][1][2] = -I; lam[6][2][1] = I;
    real r3 = 1 / sqrt((real)3);
    lam[7][0][0] = r3; lam[7][1][1] = r3; lam[7][2][2] = -2 * r3;
    for (int a = 0; a < 8; ++a)
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) TA[a][i][j] = lam[a][i][j] / 2;

    /* f^{abc} = -2 i Tr([t^a,t^b] t^c) */
    for (int a = 0; a < 8; ++a)
        for (int b = 0; b < 8; ++b)
            for (int c = 0; c < 8; ++c) {
                cplx tr = 0;
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j)
                        for (int k = 0; k < 3; ++k)
                            tr += (TA[a][i][j] * TA[b][j][k] - TA[b][i][j] * TA[a][j][k]) * TA[c][k][i];
                FABC[a][b][c] = creal(-2 * I * tr);
            }
    for (int a = 0; a < 8; ++a)
        for (int b = 0; b < 8; ++b)
            for (int c = 0; c < 8; ++c)
                for (int d = 0; d < 8; ++d) {
                    real x = 0, y = 0, z = 0;
                    for (int e = 0; e < 8; ++e) {
                        x += FABC[a][b][e] * FABC[c][d][e];
                        y += FABC[a][c][e] * FABC[b][d][e];
                        z += FABC[a][d][e] * FABC[b][c][e];
                    }
                    FF[0][a][b][c][d] = x;
                    FF[1][a][b][c][d] = y;
                    FF[2][a][b][c][d] = z;
                }
}

static void tables(void) { pthread_once(&tables_once, init_tables); }

/* ------------------------------------------------------------------------------------ */
/* Lorentz and Dirac algebra, written out with explicit matrices                         */

/* Minkowski products; no complex conjugation anywhere */
static cplx dot_cc(const cplx a[4], const cplx b[4])
{
    return a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
}
static cplx dot_cr(const cplx a[4], const real b[4])
{
    return a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
}
static real dot_rr(const real a[4], const real b[4])
{
    return a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
}

/* M = gamma^mu a_mu for a contravariant complex vector a */
static void slash_c(const cplx a[4], cplx M[4][4])
{
    cplx low[4] = {a[0], -a[1], -a[2], -a[3]};
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            cplx s = 0;
            for (int mu = 0; mu < 4; ++mu) s += GAM[mu][i][j] * low[mu];
            M[i][j] = s;
        }
}
static void slash_r(const real a[4], cplx M[4][4])
{
    cplx c[4] = {a[0], a[1], a[2], a[3]};
    slash_c(c, M);
}
static void matvec(const cplx M[4][4], const cplx x[4], cplx y[4])
{
    cplx t[4];
    for (int i = 0; i < 4; ++i) {
        cplx s = 0;
        for (int j = 0; j < 4; ++j) s += M[i][j] * x[j];
        t[i] = s;
    }
    memcpy(y, t, sizeof t);
}
/* row spinor times column spinor */
static cplx rowcol(const cplx r[4], const cplx c[4])
{
    return r[0] * c[0] + r[1] * c[1] + r[2] * c[2] + r[3] * c[3];
}
/* Dirac adjoint psibar = psi^dagger gamma^0, returned as a row */
static void dirac_bar(const cplx psi[4], cplx bar[4])
{
    for (int j = 0; j < 4; ++j) {
        cplx s = 0;
        for (int i = 0; i < 4; ++i) s += conj(psi[i]) * GAM[0][i][j];
        bar[j] = s;
    }
}
/* the vector current psibar_row gamma^mu psi (upper index mu) */
static void current(const cplx bar[4], const cplx psi[4], cplx J[4])
{
    for (int mu = 0; mu < 4; ++mu) {
        cplx t[4];
        matvec(GAM[mu], psi, t);
        J[mu] = rowcol(bar, t);
    }
}
/* quark propagator applied to a column spinor: i (qslash + m) / (q^2 - m^2) x */
static void prop_q(const real q[4], real m, const cplx x[4], cplx y[4])
{
    cplx Q[4][4];
    slash_r(q, Q);
    for (int i = 0; i < 4; ++i) Q[i][i] += m;
    cplx t[4];
    matvec(Q, x, t);
    cplx f = I / (dot_rr(q, q) - m * m);
    for (int i = 0; i < 4; ++i) y[i] = f * t[i];
}
/* quark-gluon vertex applied to a column spinor: (i g gamma^mu J_mu) x */
static void vertex_q(const cplx J[4], real g, const cplx x[4], cplx y[4])
{
    cplx S[4][4];
    slash_c(J, S);
    matvec(S, x, y);
    for (int i = 0; i < 4; ++i) y[i] *= I * g;
}

/* ------------------------------------------------------------------------------------ */
/* external states                                                                       */

/* two-component helicity eigenstates chi_lambda(p) of sigma.p/|p|; at p along -z the
 * choice chi_+ = (0,1), chi_- = (-1,0) */
static void chi(const real p[4], int lam, cplx out[2])
{
    real px = p[1], py = p[2], pz = p[3];
    real pp = sqrt(px * px + py * py + pz * pz);
    real d;
    /* d = |p| + pz, written without cancellation when pz < 0 */
    if (pz >= 0) d = pp + pz;
    else d = (px * px + py * py) / (pp - pz);
    if (!(d > 0)) {
        if (lam > 0) { out[0] = 0; out[1] = 1; }
        else { out[0] = -1; out[1] = 0; }
        return;
    }
    real nrm = sqrt(2 * pp * d);
    if (lam > 0) { out[0] = d / nrm; out[1] = (px + I * py) / nrm; }
    else { out[0] = (-px + I * py) / nrm; out[1] = d / nrm; }
}

/* omega_pm = sqrt(E pm |p|); omega_- written as m / omega_+ (exact for an on-shell p) */
static void omegas(const real p[4], real m, real *wp, real *wm)
{
    real pp = sqrt(p[1] * p[1] + p[2] * p[2] + p[3] * p[3]);
    *wp = sqrt(p[0] + pp);
    *wm = (m == 0) ? 0 : m / *wp;
}

/* u(p,lam) = (omega_{-lam} chi_lam, omega_lam chi_lam) */
static void spinor_u(const real p[4], real m, int lam, cplx u[4])
{
    cplx c[2];
    real wp, wm;
    chi(p, lam, c);
    omegas(p, m, &wp, &wm);
    real up = (lam > 0) ? wm : wp, lo = (lam > 0) ? wp : wm;
    u[0] = up * c[0]; u[1] = up * c[1];
    u[2] = lo * c[0]; u[3] = lo * c[1];
}
/* v(p,lam) = (-lam omega_lam chi_{-lam}, lam omega_{-lam} chi_{-lam}) */
static void spinor_v(const real p[4], real m, int lam, cplx v[4])
{
    cplx c[2];
    real wp, wm;
    chi(p, -lam, c);
    omegas(p, m, &wp, &wm);
    real wl = (lam > 0) ? wp : wm, wml = (lam > 0) ? wm : wp;
    v[0] = -lam * wl * c[0]; v[1] = -lam * wl * c[1];
    v[2] = lam * wml * c[0]; v[3] = lam * wml * c[1];
}
/* spin along z in the rest frame, boosted: u = (sqrt(p.sigma) xi, sqrt(p.sigmabar) xi),
 * v = (sqrt(p.sigma) eta, -sqrt(p.sigmabar) eta), sqrt(p.sigma) = (p.sigma + m)/sqrt(2(E+m)),
 * xi, eta = (1,0) for s = +1 and (0,1) for s = -1.  Massive particles only. */
static void spinor_z(const real p[4], real m, int s, int is_v, cplx out[4])
{
    real E = p[0], px = p[1], py = p[2], pz = p[3];
    cplx ps[2][2] = {{E - pz, -(px - I * py)}, {-(px + I * py), E + pz}};   /* p.sigma    */
    cplx pb[2][2] = {{E + pz, px - I * py}, {px + I * py, E - pz}};         /* p.sigmabar */
    real nrm = sqrt(2 * (E + m));
    cplx xi[2] = {(s > 0) ? 1 : 0, (s > 0) ? 0 : 1};
    for (int i = 0; i < 2; ++i) {
        cplx a = 0, b = 0;
        for (int j = 0; j < 2; ++j) {
            a += (ps[i][j] + (i == j ? m : 0)) * xi[j];
            b += (pb[i][j] + (i == j ? m : 0)) * xi[j];
        }
        out[i] = a / nrm;
        out[i + 2] = (is_v ? -b : b) / nrm;
    }
}

/* eps(k,lam) = (-lam eps1 - i eps2)/sqrt2 with eps1 = (0, cos th cos ph, cos th sin ph,
 * -sin th), eps2 = (0, -sin ph, cos ph, 0); complex conjugate for an outgoing gluon.
 * basis 1: the linear polarisations eps1 (lam=+1) and eps2 (lam=-1). */
static void polvec(const real k[4], int lam, int outgoing, int basis, cplx e[4])
{
    real kx = k[1], ky = k[2], kz = k[3];
    real kt = sqrt(kx * kx + ky * ky);
    real kk = sqrt(kt * kt + kz * kz);
    real ct = kz / kk, st = kt / kk;
    real cp = 1, sp = 0;
    if (kt > 0) { cp = kx / kt; sp = ky / kt; }
    real e1[4] = {0, ct * cp, ct * sp, -st};
    real e2[4] = {0, -sp, cp, 0};
    if (basis == 1) {
        for (int mu = 0; mu < 4; ++mu) e[mu] = (lam > 0) ? e1[mu] : e2[mu];
        return;
    }
    real r2 = sqrt((real)2);
    for (int mu = 0; mu < 4; ++mu) {
        cplx x = (-lam * e1[mu] - I * e2[mu]) / r2;
        e[mu] = outgoing ? conj(x) : x;
    }
}

/* ------------------------------------------------------------------------------------ */
/* the two vertex functions of the gluon recursion                                        */

/* three-gluon vertex with the off-shell leg's incoming momentum -(P1+P2):
 * V^mu = (J1.J2)(P1-P2)^mu + J2^mu J1.(P1+2P2) - J1^mu J2.(2P1+P2) */
static void vvv(const cplx J1[4], const real P1[4], const cplx J2[4], const real P2[4], cplx V[4])
{
    real a[4], b[4], c[4];
    for (int mu = 0; mu < 4; ++mu) {
        a[mu] = P1[mu] - P2[mu];
        b[mu] = P1[mu] + 2 * P2[mu];
        c[mu] = 2 * P1[mu] + P2[mu];
    }
    cplx d12 = dot_cc(J1, J2), d1b = dot_cr(J1, b), d2c = dot_cr(J2, c);
    for (int mu = 0; mu < 4; ++mu) V[mu] = d12 * a[mu] + J2[mu] * d1b - J1[mu] * d2c;
}
/* colour-ordered four-gluon vertex for ordered X, Y, Z: 2(X.Z)Y - (X.Y)Z - (Y.Z)X */
static void vvvv_ordered(const cplx X[4], const cplx Y[4], const cplx Z[4], cplx W[4])
{
    cplx xz = dot_cc(X, Z), xy = dot_cc(X, Y), yz = dot_cc(Y, Z);
    for (int mu = 0; mu < 4; ++mu) W[mu] = 2 * xz * Y[mu] - xy * Z[mu] - yz * X[mu];
}

/* ------------------------------------------------------------------------------------ */
/* process set-up: external wavefunctions for one helicity                                */

typedef struct {
    int ng;               /* gluons                                                     */
    real q[NG_MAX][4];    /* gluon momenta, counted incoming (k or -k)                  */
    real k[NG_MAX][4];    /* gluon physical momenta                                     */
    cplx e[NG_MAX][4];    /* polarisations (eps for incoming, eps^* for outgoing)       */
    int gpar[NG_MAX];     /* particle index of each gluon                                */
    cplx ubar[4];         /* outgoing quark, row spinor                                 */
    cplx v[4];            /* outgoing antiquark, column spinor                          */
    real pq[4], pa[4];    /* quark and antiquark momenta                                */
    real m, g;
} ext_t;

static int helicity_of(int n_par, int h, int i) { return ((h >> (n_par - 1 - i)) & 1) ? 1 : -1; }

/* QCD processes: particles (g, g, t, t~, g, ...); gg->gg: (g, g, g, g). */
static void setup_qcd(int proc, const double *p, const real *par, int h, int basis, ext_t *X)
{
    int n_par = N_PAR[proc];
    real m = par[0], gs = sqrt(4 * PI_R * par[2]);
    X->m = m;
    X->g = gs;
    int ng = 0;
    for (int i = 0; i < n_par; ++i) {
        int is_gluon = (proc == P_GG_GG) || (i != 2 && i != 3);
        real pi[4] = {p[4 * i], p[4 * i + 1], p[4 * i + 2], p[4 * i + 3]};
        int lam = helicity_of(n_par, h, i);
        if (is_gluon) {
            int outgoing = (i >= 2);
            for (int mu = 0; mu < 4; ++mu) {
                X->k[ng][mu] = pi[mu];
                X->q[ng][mu] = outgoing ? -pi[mu] : pi[mu];
            }
            polvec(pi, lam, outgoing, basis, X->e[ng]);
            X->gpar[ng] = i;
            ++ng;
        } else if (i == 2) {
            cplx u[4];
            if (basis == 1) spinor_z(pi, m, lam, 0, u);
            else spinor_u(pi, m, lam, u);
            dirac_bar(u, X->ubar);
            memcpy(X->pq, pi, sizeof pi);
        } else {
            if (basis == 1) spinor_z(pi, m, lam, 1, X->v);
            else spinor_v(pi, m, lam, X->v);
            memcpy(X->pa, pi, sizeof pi);
        }
    }
    X->ng = ng;
}

/* ------------------------------------------------------------------------------------ */
/* colour-ordered Berends-Giele recursion                                                 */

/* Off-shell colour-ordered gluon currents Jh[a][b] for the contiguous runs
 * s[a..b] of the ordered gluon list s (length n), with their summed momenta P[a][b].
 * Jh of a single gluon is its polarisation; a longer run sums the three-gluon vertex
 * over its two-way splits (factor -g) and the four-gluon vertex over its three-way
 * splits (factor +g^2), divided by P^2.  These two factors are the Feynman rules above
 * after f^{abc} t^c = -i [t^a, t^b] and the -i of the propagator are absorbed.  With
 * amputate_full the full run is left without the 1/P^2. */
static void bg_gluon_currents(const ext_t *X, const int *s, int n, int amputate_full,
                              cplx Jh[NG_MAX][NG_MAX][4], real P[NG_MAX][NG_MAX][4])
{
    real g = X->g;
    for (int len = 1; len <= n; ++len)
        for (int a = 0; a + len - 1 < n; ++a) {
            int b = a + len - 1;
            for (int mu = 0; mu < 4; ++mu) {
                real t = 0;
                for (int k = a; k <= b; ++k) t += X->q[s[k]][mu];
                P[a][b][mu] = t;
            }
            if (len == 1) {
                memcpy(Jh[a][a], X->e[s[a]], sizeof(cplx) * 4);
                continue;
            }
            cplx acc[4] = {0, 0, 0, 0};
            for (int k = a; k < b; ++k) {
                cplx V[4];
                vvv(Jh[a][k], P[a][k], Jh[k + 1][b], P[k + 1][b], V);
                for (int mu = 0; mu < 4; ++mu) acc[mu] += -g * V[mu];
            }
            for (int k = a; k < b; ++k)
                for (int l = k + 1; l < b; ++l) {
                    cplx W[4];
                    vvvv_ordered(Jh[a][k], Jh[k + 1][l], Jh[l + 1][b], W);
                    for (int mu = 0; mu < 4; ++mu) acc[mu] += g * g * W[mu];
                }
            real den = (amputate_full && len == n) ? 1 : dot_rr(P[a][b], P[a][b]);
            for (int mu = 0; mu < 4; ++mu) Jh[a][b][mu] = acc[mu] / den;
        }
}

/* A(sigma) for one quark line: ubar(p_q) ... v(p_a) with the gluons attached in the
 * order s[0] (next to the quark) .. s[n-1] (next to the antiquark).  The antiquark-side
 * strings psi[a] absorb the runs s[a..]; the momentum on the propagator before psi[a]
 * is -p_a + sum of the absorbed gluon momenta. */
static cplx bg_qline(const ext_t *X, const int *s)
{
    int n = X->ng;
    cplx Jh[NG_MAX][NG_MAX][4];
    real P[NG_MAX][NG_MAX][4];
    bg_gluon_currents(X, s, n, 0, Jh, P);
    cplx psi[NG_MAX + 1][4];
    memcpy(psi[n], X->v, sizeof(cplx) * 4);
    for (int a = n - 1; a >= 1; --a) {
        cplx acc[4] = {0, 0, 0, 0};
        for (int k = a; k < n; ++k) {
            cplx t[4];
            vertex_q(Jh[a][k], X->g, psi[k + 1], t);
            for (int i = 0; i < 4; ++i) acc[i] += t[i];
        }
        real q[4];
        for (int mu = 0; mu < 4; ++mu) q[mu] = -X->pa[mu] + P[a][n - 1][mu];
        prop_q(q, X->m, acc, psi[a]);
    }
    cplx amp = 0;
    for (int k = 0; k < n; ++k) {
        cplx t[4];
        vertex_q(Jh[0][k], X->g, psi[k + 1], t);
        amp += rowcol(X->ubar, t);
    }
    return amp;
}

/* pure gluons: A(pi) = 2 eps_last . Vhat(pi), Vhat the amputated current of the other
 * gluons in the order pi, so that M = sum_pi Tr(t^{a_last} t^{a_pi1} ...) A(pi).  The
 * recursion's full run is i times the vertex sum above (its current is -i/P^2 times the
 * vertex sum), hence the factor i. */
static cplx bg_gluons(const ext_t *X, const int *s)
{
    int n = X->ng - 1;
    cplx Jh[NG_MAX][NG_MAX][4];
    real P[NG_MAX][NG_MAX][4];
    bg_gluon_currents(X, s, n, 1, Jh, P);
    return 2 * I * dot_cc(X->e[X->ng - 1], Jh[0][n - 1]);
}

/* ------------------------------------------------------------------------------------ */
/* permutations and colour matrices                                                      */

static int factorial(int n) { int f = 1; for (int i = 2; i <= n; ++i) f *= i; return f; }

/* all permutations of 0..n-1 in lexicographic order */
static int perm_list(int n, int out[][NG_MAX])
{
    int a[NG_MAX];
    for (int i = 0; i < n; ++i) a[i] = i;
    int cnt = 0;
    for (;;) {
        memcpy(out[cnt++], a, sizeof(int) * NG_MAX);
        int i = n - 2;
        while (i >= 0 && a[i] > a[i + 1]) --i;
        if (i < 0) break;
        int j = n - 1;
        while (a[j] < a[i]) --j;
        int t = a[i]; a[i] = a[j]; a[j] = t;
        for (int l = i + 1, r = n - 1; l < r; ++l, --r) { t = a[l]; a[l] = a[r]; a[r] = t; }
    }
    return cnt;
}

static void mat3_mul(const cplx A[3][3], const cplx B[3][3], cplx C[3][3])
{
    cplx T[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cplx s = 0;
            for (int k = 0; k < 3; ++k) s += A[i][k] * B[k][j];
            T[i][j] = s;
        }
    memcpy(C, T, sizeof T);
}

/* product t^{col[s[0]]} t^{col[s[1]]} ... */
static void tstring(const int *col, const int *s, int n, cplx out[3][3])
{
    memcpy(out, TA[col[s[0]]], sizeof(cplx) * 9);
    for (int k = 1; k < n; ++k) mat3_mul(out, TA[col[s[k]]], out);
}

/* Quark-line colour matrix by its definition, C[s][t] = sum over all gluon colours and
 * the two quark indices of (T^s)_{ij} conj((T^t)_{ij}); cost 8^n n!^2. */
static void colour_matrix_q_direct(int n, real *C)
{
    int perms[NPERM_MAX][NG_MAX];
    int np = perm_list(n, perms);
    cplx (*T)[3][3] = malloc(sizeof(cplx) * 9 * np);
    memset(C, 0, sizeof(real) * np * np);
    int ncol = 1;
    for (int i = 0; i < n; ++i) ncol *= 8;
    for (int c = 0; c < ncol; ++c) {
        int col[NG_MAX];
        for (int i = 0, x = c; i < n; ++i, x /= 8) col[i] = x % 8;
        for (int s = 0; s < np; ++s) tstring(col, perms[s], n, T[s]);
        for (int s = 0; s < np; ++s)
            for (int t = 0; t < np; ++t) {
                cplx acc = 0;
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) acc += T[s][i][j] * conj(T[t][i][j]);
                C[s * np + t] += creal(acc);
            }
    }
    free(T);
}

/* The same matrix with the summed colour labels renamed: C[s][t] = c(s^-1 t) with
 * c(r) = sum_colours sum_ij (T^id)_{ij} conj((T^r)_{ij}); cost 8^n n!. */
static void colour_matrix_q_relabel(int n, real *C)
{
    int perms[NPERM_MAX][NG_MAX];
    int np = perm_list(n, perms);
    real c[NPERM_MAX];
    memset(c, 0, sizeof c);
    int ncol = 1;
    for (int i = 0; i < n; ++i) ncol *= 8;
    for (int cc = 0; cc < ncol; ++cc) {
        int col[NG_MAX];
        for (int i = 0, x = cc; i < n; ++i, x /= 8) col[i] = x % 8;
        cplx T0[3][3];
        tstring(col, perms[0], n, T0);
        for (int r = 0; r < np; ++r) {
            cplx Tr[3][3];
            tstring(col, perms[r], n, Tr);
            cplx acc = 0;
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) acc += T0[i][j] * conj(Tr[i][j]);
            c[r] += creal(acc);
        }
    }
    for (int s = 0; s < np; ++s)
        for (int t = 0; t < np; ++t) {
            int inv[NG_MAX], r[NG_MAX];
            for (int k = 0; k < n; ++k) inv[perms[s][k]] = k;
            for (int k = 0; k < n; ++k) r[k] = inv[perms[t][k]];
            int idx = -1;
            for (int q = 0; q < np && idx < 0; ++q)
                if (memcmp(perms[q], r, sizeof(int) * n) == 0) idx = q;
            C[s * np + t] = c[idx];
        }
}

/* Single-trace colour matrix for n gluons with the last fixed:
 * C[s][t] = sum_colours Tr(t^{a_n} T^s) conj(Tr(t^{a_n} T^t)), s, t orderings of the
 * first n-1 gluons. */
static void colour_matrix_g_direct(int n, real *C)
{
    int perms[NPERM_MAX][NG_MAX];
    int np = perm_list(n - 1, perms);
    cplx tr[NPERM_MAX];
    memset(C, 0, sizeof(real) * np * np);
    int ncol = 1;
    for (int i = 0; i < n; ++i) ncol *= 8;
    for (int cc = 0; cc < ncol; ++cc) {
        int col[NG_MAX];
        for (int i = 0, x = cc; i < n; ++i, x /= 8) col[i] = x % 8;
        for (int s = 0; s < np; ++s) {
            cplx T[3][3];
            tstring(col, perms[s], n - 1, T);
            cplx acc = 0;
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) acc += TA[col[n - 1]][i][j] * T[j][i];
            tr[s] = acc;
        }
        for (int s = 0; s < np; ++s)
            for (int t = 0; t < np; ++t) C[s * np + t] += creal(tr[s] * conj(tr[t]));
    }
}

/* cached colour matrices: kind 0 quark line with n = 2..5 gluons, kind 1 single trace
 * with n = 4 gluons */
static real *CMAT[2][NG_MAX + 1];
static pthread_mutex_t cmat_lock = PTHREAD_MUTEX_INITIALIZER;

static const real *colour_matrix(int kind, int n)
{
    tables();
    pthread_mutex_lock(&cmat_lock);
    if (!CMAT[kind][n]) {
        int np = factorial(kind == 0 ? n : n - 1);
        real *C = malloc(sizeof(real) * np * np);
        if (kind == 1) colour_matrix_g_direct(n, C);
        else if (n <= 4) colour_matrix_q_direct(n, C);
        else colour_matrix_q_relabel(n, C);
        CMAT[kind][n] = C;
    }
    pthread_mutex_unlock(&cmat_lock);
    return CMAT[kind][n];
}

/* ------------------------------------------------------------------------------------ */
/* e+ e- -> mu+ mu- through one photon: particles (e+, e-, mu+, mu-).
 * M = [vbar(p1) (i e gamma^mu) u(p2)] (-i g_{mu nu}/s) [ubar(p4) (i e gamma^nu) v(p3)] */
static cplx amp_eemumu(const double *p, const real *par, int h, int basis)
{
    (void)basis;
    real e = sqrt(4 * PI_R * par[1]);
    real p1[4], p2[4], p3[4], p4[4];
    for (int mu = 0; mu < 4; ++mu) {
        p1[mu] = p[mu]; p2[mu] = p[4 + mu]; p3[mu] = p[8 + mu]; p4[mu] = p[12 + mu];
    }
    cplx v1[4], v1bar[4], u2[4], v3[4], u4[4], u4bar[4];
    spinor_v(p1, 0, helicity_of(4, h, 0), v1);
    dirac_bar(v1, v1bar);
    spinor_u(p2, 0, helicity_of(4, h, 1), u2);
    spinor_v(p3, 0, helicity_of(4, h, 2), v3);
    spinor_u(p4, 0, helicity_of(4, h, 3), u4);
    dirac_bar(u4, u4bar);
    cplx Je[4], Jm[4];
    current(v1bar, u2, Je);
    current(u4bar, v3, Jm);
    real P[4];
    for (int mu = 0; mu < 4; ++mu) P[mu] = p1[mu] + p2[mu];
    real s = dot_rr(P, P);
    return (I * e) * (I * e) * (-I / s) * dot_cc(Je, Jm);
}

/* e+ e- -> mu+ mu- with photon and Z exchange (Peskin & Schroeder's electroweak vertices):
 * photon -i e Q gamma^mu, Z -i (g / cos theta_W) gamma^mu (T3 P_L - Q sin^2 theta_W) with
 * P_L = (1 - gamma5)/2, g = e / sin theta_W; propagators -i g_{mu nu} / s and
 * -i g_{mu nu} / (s - M_Z^2 + i M_Z Gamma_Z) (the k_mu k_nu term vanishes between massless
 * currents).  For e and mu: Q = -1, T3 = -1/2.  gamma5 is diag(-1, -1, 1, 1) in this
 * representation. */
static cplx amp_eemumu_z(const double *p, const real *par, int h, int diagram_mask)
{
    real e = sqrt(4 * PI_R * par[1]);
    real sw2 = 1 - EW_MW * EW_MW / (EW_MZ * EW_MZ), cw2 = 1 - sw2;
    real gz = e / sqrt(sw2 * cw2);
    real cl = -0.5 + sw2, cr = sw2;              /* T3 - Q sw2 on P_L; -Q sw2 on P_R */
    real p1[4], p2[4], p3[4], p4[4];
    for (int mu = 0; mu < 4; ++mu) {
        p1[mu] = p[mu]; p2[mu] = p[4 + mu]; p3[mu] = p[8 + mu]; p4[mu] = p[12 + mu];
    }
    cplx v1[4], v1bar[4], u2[4], v3[4], u4[4], u4bar[4];
    spinor_v(p1, 0, helicity_of(4, h, 0), v1);
    dirac_bar(v1, v1bar);
    spinor_u(p2, 0, helicity_of(4, h, 1), u2);
    spinor_v(p3, 0, helicity_of(4, h, 2), v3);
    spinor_u(p4, 0, helicity_of(4, h, 3), u4);
    dirac_bar(u4, u4bar);
    /* chiral projections of the column spinors: P_L keeps components 0, 1 */
    cplx u2L[4] = {u2[0], u2[1], 0, 0}, u2R[4] = {0, 0, u2[2], u2[3]};
    cplx v3L[4] = {v3[0], v3[1], 0, 0}, v3R[4] = {0, 0, v3[2], v3[3]};
    cplx Je[4], Jm[4], JeL[4], JeR[4], JmL[4], JmR[4], JeZ[4], JmZ[4];
    current(v1bar, u2, Je);
    current(u4bar, v3, Jm);
    current(v1bar, u2L, JeL);
    current(v1bar, u2R, JeR);
    current(u4bar, v3L, JmL);
    current(u4bar, v3R, JmR);
    for (int mu = 0; mu < 4; ++mu) {
        JeZ[mu] = cl * JeL[mu] + cr * JeR[mu];
        JmZ[mu] = cl * JmL[mu] + cr * JmR[mu];
    }
    real P[4];
    for (int mu = 0; mu < 4; ++mu) P[mu] = p1[mu] + p2[mu];
    real s = dot_rr(P, P);
    cplx a = 0;
    if (diagram_mask & 1) a += (-I * e * -1) * (-I * e * -1) * (-I / s) * dot_cc(Je, Jm);
    if (diagram_mask & 2)
        a += (-I * gz) * (-I * gz) * (-I / (s - EW_MZ * EW_MZ + I * EW_MZ * EW_WZ)) * dot_cc(JeZ, JmZ);
    return a;
}

/* ------------------------------------------------------------------------------------ */
/* colour-ordered amplitudes and the colour-summed |M_h|^2                               */

static int n_gluons(int proc) { return proc == P_GG_GG ? 4 : N_PAR[proc] - 2; }

/* all colour-ordered amplitudes of helicity h, in lexicographic permutation order;
 * gauge_gluon >= 0 replaces that gluon's polarisation by its physical momentum. */
static int partials(int proc, const double *p, const real *par, int h, int basis,
                    int gauge_gluon, cplx *A)
{
    tables();
    ext_t X;
    setup_qcd(proc, p, par, h, basis, &X);
    if (gauge_gluon >= 0)
        for (int mu = 0; mu < 4; ++mu) X.e[gauge_gluon][mu] = X.k[gauge_gluon][mu];
    int perms[NPERM_MAX][NG_MAX];
    int n = n_gluons(proc);
    int np;
    if (proc == P_GG_GG) {
        np = perm_list(n - 1, perms);
        for (int s = 0; s < np; ++s) A[s] = bg_gluons(&X, perms[s]);
    } else {
        np = perm_list(n, perms);
        for (int s = 0; s < np; ++s) A[s] = bg_qline(&X, perms[s]);
    }
    return np;
}

static real me_helicity(int proc, const double *p, const real *par, int h, int basis)
{
    if (proc == P_EE_MUMU) {
        cplx a = amp_eemumu(p, par, h, basis);
        return creal(a * conj(a));
    }
    if (proc == P_EE_MUMU_Z) {
        cplx a = amp_eemumu_z(p, par, h, 3);
        return creal(a * conj(a));
    }
    cplx A[NPERM_MAX];
    int np = partials(proc, p, par, h, basis, -1, A);
    const real *C = colour_matrix(proc == P_GG_GG ? 1 : 0, n_gluons(proc));
    real sum = 0;
    for (int s = 0; s < np; ++s) {
        cplx row = 0;
        for (int t = 0; t < np; ++t) row += C[s * np + t] * A[t];
        sum += creal(conj(A[s]) * row);
    }
    return sum;
}

/* ------------------------------------------------------------------------------------ */
/* colour-dressed recursion with explicit colours (brute force)                         */

typedef struct {
    cplx J[32][8][4];    /* dressed current of each gluon subset, per adjoint colour    */
    int nz[32][8];
    real P[32][4];
} dressed_t;

static int lowbit(int S) { return S & -S; }

/* Colour-dressed gluon currents for all subsets of the n gluons with external colours
 * col[]; the subset `amp_set` (if nonzero) is left without its propagator.  Each
 * unordered split is counted once: the first part holds the lowest gluon of S. */
static void dressed_currents(const ext_t *X, int n, const int *col, int amp_set, dressed_t *D)
{
    real g = X->g;
    int full = (1 << n) - 1;
    for (int S = 1; S <= full; ++S) {
        for (int mu = 0; mu < 4; ++mu) {
            real t = 0;
            for (int i = 0; i < n; ++i)
                if (S >> i & 1) t += X->q[i][mu];
            D->P[S][mu] = t;
        }
        memset(D->J[S], 0, sizeof D->J[S]);
        memset(D->nz[S], 0, sizeof D->nz[S]);
        if ((S & (S - 1)) == 0) {
            int i = __builtin_ctz(S);
            memcpy(D->J[S][col[i]], X->e[i], sizeof(cplx) * 4);
            D->nz[S][col[i]] = 1;
            continue;
        }
        cplx acc[8][4];
        memset(acc, 0, sizeof acc);
        int lo = lowbit(S);
        /* three-gluon vertex g f^{abc} [..] with legs (a: off-shell, b: S1, c: S2) */
        for (int S1 = (S - 1) & S; S1; S1 = (S1 - 1) & S) {
            if (!(S1 & lo)) continue;
            int S2 = S ^ S1;
            for (int b = 0; b < 8; ++b) {
                if (!D->nz[S1][b]) continue;
                for (int c = 0; c < 8; ++c) {
                    if (!D->nz[S2][c]) continue;
                    cplx V[4];
                    vvv(D->J[S1][b], D->P[S1], D->J[S2][c], D->P[S2], V);
                    for (int a = 0; a < 8; ++a) {
                        real f = FABC[a][b][c];
                        if (f == 0) continue;
                        for (int mu = 0; mu < 4; ++mu) acc[a][mu] += g * f * V[mu];
                    }
                }
            }
        }
        /* four-gluon vertex -i g^2 [f^{abe}f^{cde}(g^{mu rho}g^{nu sigma} - g^{mu sigma}g^{nu rho})
         * + f^{ace}f^{bde}(g^{mu nu}g^{rho sigma} - g^{mu sigma}g^{nu rho})
         * + f^{ade}f^{bce}(g^{mu nu}g^{rho sigma} - g^{mu rho}g^{nu sigma})], legs (a,mu) off-shell,
         * (b,nu) S1, (c,rho) S2, (d,sigma) S3 */
        for (int S1 = (S - 1) & S; S1; S1 = (S1 - 1) & S) {
            if (!(S1 & lo)) continue;
            int R = S ^ S1;
            int lo2 = lowbit(R);
            for (int S2 = (R - 1) & R; S2; S2 = (S2 - 1) & R) {
                if (!(S2 & lo2)) continue;
                int S3 = R ^ S2;
                for (int b = 0; b < 8; ++b) {
                    if (!D->nz[S1][b]) continue;
                    for (int c = 0; c < 8; ++c) {
                        if (!D->nz[S2][c]) continue;
                        for (int d = 0; d < 8; ++d) {
                            if (!D->nz[S3][d]) continue;
                            const cplx *J1 = D->J[S1][b], *J2 = D->J[S2][c], *J3 = D->J[S3][d];
                            cplx d12 = dot_cc(J1, J2), d13 = dot_cc(J1, J3), d23 = dot_cc(J2, J3);
                            cplx L1[4], L2[4], L3[4];
                            for (int mu = 0; mu < 4; ++mu) {
                                L1[mu] = J2[mu] * d13 - J3[mu] * d12;
                                L2[mu] = J1[mu] * d23 - J3[mu] * d12;
                                L3[mu] = J1[mu] * d23 - J2[mu] * d13;
                            }
                            for (int a = 0; a < 8; ++a) {
                                real f1 = FF[0][a][b][c][d], f2 = FF[1][a][b][c][d], f3 = FF[2][a][b][c][d];
                                if (f1 == 0 && f2 == 0 && f3 == 0) continue;
                                for (int mu = 0; mu < 4; ++mu)
                                    acc[a][mu] += -I * g * g * (f1 * L1[mu] + f2 * L2[mu] + f3 * L3[mu]);
                            }
                        }
                    }
                }
            }
        }
        cplx f = (S == amp_set) ? 1 : -I / dot_rr(D->P[S], D->P[S]);
        for (int a = 0; a < 8; ++a) {
            int any = 0;
            for (int mu = 0; mu < 4; ++mu) {
                D->J[S][a][mu] = f * acc[a][mu];
                if (acc[a][mu] != 0) any = 1;
            }
            D->nz[S][a] = any;
        }
    }
}

/* Full amplitude with explicit colours for one quark line: out[i] for quark colour i,
 * antiquark colour j.  psi[R][k] is the antiquark-side spinor with gluon set R absorbed,
 * colour index k; the block R1 next to the quark side is summed over all subsets. */
static void dressed_qline(const ext_t *X, const dressed_t *D, int j, cplx out[3])
{
    int n = X->ng, full = (1 << n) - 1;
    static __thread cplx psi[32][3][4];
    memset(psi[0], 0, sizeof psi[0]);
    memcpy(psi[0][j], X->v, sizeof(cplx) * 4);
    for (int R = 1; R <= full; ++R) {
        cplx acc[3][4];
        memset(acc, 0, sizeof acc);
        for (int R1 = R; R1; R1 = (R1 - 1) & R) {
            int rest = R ^ R1;
            for (int a = 0; a < 8; ++a) {
                if (!D->nz[R1][a]) continue;
                for (int k = 0; k < 3; ++k) {
                    cplx t[4];
                    vertex_q(D->J[R1][a], X->g, psi[rest][k], t);
                    for (int i = 0; i < 3; ++i) {
                        cplx c = TA[a][i][k];
                        if (c == 0) continue;
                        for (int l = 0; l < 4; ++l) acc[i][l] += c * t[l];
                    }
                }
            }
        }
        if (R == full) {
            for (int i = 0; i < 3; ++i) out[i] = rowcol(X->ubar, acc[i]);
        } else {
            real q[4];
            for (int mu = 0; mu < 4; ++mu) q[mu] = -X->pa[mu] + D->P[R][mu];
            for (int i = 0; i < 3; ++i) prop_q(q, X->m, acc[i], psi[R][i]);
        }
    }
}

/* ------------------------------------------------------------------------------------ */
/* exported API (names are the same in the double and the long double build)            */

int or_n_par(int proc) { return (proc >= 0 && proc < N_PROC) ? N_PAR[proc] : -1; }
int or_n_colour_orderings(int proc)
{
    if (proc < 0 || proc >= N_PROC) return -1;
    if (is_ee(proc)) return 1;
    return factorial(proc == P_GG_GG ? 3 : n_gluons(proc));
}
int or_real_bytes(void) { return (int)sizeof(real); }

static void load_par(const double *params, real par[3])
{
    for (int i = 0; i < 3; ++i) par[i] = params[i];
}

/* averaged sum over all helicities and colours; params = {m_t, alpha_em, alpha_s};
 * me_hel (optional) receives the colour-summed |M_h|^2 of every helicity */
/* ee -> mumu with Z: the amplitude of helicity h from the diagrams in `mask` (1 photon,
 * 2 Z, 3 both) */
int or_ee_z_amp(const double *params, const double *p, int h, int mask, double *out)
{
    tables();
    real par[3];
    load_par(params, par);
    cplx a = amp_eemumu_z(p, par, h, mask);
    out[0] = (double)creal(a);
    out[1] = (double)cimag(a);
    return 0;
}

double or_me(int proc, const double *params, const double *p, int basis, double *me_hel)
{
    if (proc < 0 || proc >= N_PROC) return -1;
    tables();
    real par[3];
    load_par(params, par);
    int n_par = N_PAR[proc];
    int nh = 1 << n_par;
    real sum = 0;
    for (int h = 0; h < nh; ++h) {
        real x = me_helicity(proc, p, par, h, basis);
        if (me_hel) me_hel[h] = (double)x;
        sum += x;
    }
    real avg = is_ee(proc) ? 4 : 256;
    return (double)(sum / avg);
}

/* batch form: p[n_evt][n_par][4] -> me[n_evt] */
int or_me_batch(int proc, const double *params, const double *p, int64_t n_evt, int basis,
                double *me)
{
    if (proc < 0 || proc >= N_PROC || n_evt < 0) return -1;
    int n_par = N_PAR[proc];
    for (int64_t e = 0; e < n_evt; ++e)
        me[e] = or_me(proc, params, p + (size_t)e * n_par * 4, basis, NULL);
    return 0;
}

/* colour-ordered amplitudes (re, im interleaved) of helicity h; returns their number */
int or_partials(int proc, const double *params, const double *p, int h, int basis,
                int gauge_gluon, double *out)
{
    if (!is_qcd(proc)) return -1;
    real par[3];
    load_par(params, par);
    cplx A[NPERM_MAX];
    int np = partials(proc, p, par, h, basis, gauge_gluon, A);
    for (int s = 0; s < np; ++s) {
        out[2 * s] = (double)creal(A[s]);
        out[2 * s + 1] = (double)cimag(A[s]);
    }
    return np;
}

/* the permutations that label the colour orderings, lexicographic */
int or_orderings(int proc, int *out)
{
    if (!is_qcd(proc)) return -1;
    int perms[NPERM_MAX][NG_MAX];
    int n = (proc == P_GG_GG) ? 3 : n_gluons(proc);
    int np = perm_list(n, perms);
    for (int s = 0; s < np; ++s)
        for (int k = 0; k < n; ++k) out[s * n + k] = perms[s][k];
    return np;
}

int or_colour_matrix(int proc, double *out)
{
    if (!is_qcd(proc)) return -1;
    int kind = (proc == P_GG_GG) ? 1 : 0;
    int n = n_gluons(proc);
    int np = factorial(kind ? n - 1 : n);
    const real *C = colour_matrix(kind, n);
    for (int i = 0; i < np * np; ++i) out[i] = (double)C[i];
    return np;
}

/* quark-line colour matrix computed both by definition and by relabelling (n <= 4) */
int or_colour_matrix_methods(int n, double *direct, double *relabel)
{
    if (n < 1 || n > 4) return -1;
    tables();
    int np = factorial(n);
    real *a = malloc(sizeof(real) * np * np), *b = malloc(sizeof(real) * np * np);
    colour_matrix_q_direct(n, a);
    colour_matrix_q_relabel(n, b);
    for (int i = 0; i < np * np; ++i) { direct[i] = (double)a[i]; relabel[i] = (double)b[i]; }
    free(a);
    free(b);
    return np;
}

/* Full amplitude for helicity h and explicit colours, two ways:
 *   dressed: the colour-dressed recursion (explicit f^{abc}, t^a);
 *   decomposed: sum over orderings of the colour factor times A(sigma).
 * colours = {a_gluon_0, .., a_gluon_{ng-1}, i_quark, j_antiquark} (QCD with quarks) or
 * {a_0, .., a_3} (gg -> gg); gluons counted in particle order. */
int or_amp_explicit_colour(int proc, const double *params, const double *p, int h,
                           const int *colours, double *dressed, double *decomposed)
{
    if (!is_qcd(proc)) return -1;
    tables();
    real par[3];
    load_par(params, par);
    ext_t X;
    setup_qcd(proc, p, par, h, 0, &X);
    int n = X.ng;
    static __thread dressed_t D;
    cplx md, mc = 0;
    cplx A[NPERM_MAX];
    int perms[NPERM_MAX][NG_MAX];
    if (proc == P_GG_GG) {
        int amp_set = (1 << (n - 1)) - 1;
        dressed_currents(&X, n - 1, colours, amp_set, &D);
        md = dot_cc(D.J[amp_set][colours[n - 1]], X.e[n - 1]);
        int np = perm_list(n - 1, perms);
        for (int s = 0; s < np; ++s) A[s] = bg_gluons(&X, perms[s]);
        for (int s = 0; s < np; ++s) {
            cplx T[3][3];
            tstring(colours, perms[s], n - 1, T);
            cplx tr = 0;
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) tr += TA[colours[n - 1]][i][j] * T[j][i];
            mc += tr * A[s];
        }
    } else {
        dressed_currents(&X, n, colours, 0, &D);
        cplx out[3];
        dressed_qline(&X, &D, colours[n + 1], out);
        md = out[colours[n]];
        int np = perm_list(n, perms);
        for (int s = 0; s < np; ++s) A[s] = bg_qline(&X, perms[s]);
        for (int s = 0; s < np; ++s) {
            cplx T[3][3];
            tstring(colours, perms[s], n, T);
            mc += T[colours[n]][colours[n + 1]] * A[s];
        }
    }
    dressed[0] = (double)creal(md); dressed[1] = (double)cimag(md);
    decomposed[0] = (double)creal(mc); decomposed[1] = (double)cimag(mc);
    return 0;
}

/* Colour-stripped amplitude of ONE Feynman diagram of a quark-line process, helicity h
 * (for the single-diagram channel weights).  The diagram is a postfix program:
 *   op >= 0      push gluon op's polarisation (gluons counted in particle order)
 *   op == -1     pop B, pop A, push the three-gluon current  g V(A, B) (-i / P^2)
 *                (the Lorentz part of g f^{abc}[..] with a off-shell, b = A, c = B)
 *   op == -2-s   pop C, B, A, push the four-gluon current of colour structure s = 0, 1, 2:
 *                -i g^2 L_s(A, B, C) (-i / P^2), L_0 = B(A.C) - C(A.B), L_1 = A(B.C) - C(A.B),
 *                L_2 = A(B.C) - B(A.C), paired with f^{abe}f^{cde}, f^{ace}f^{bde}, f^{ade}f^{bce}
 *   op == -10-k  the k currents on top of the stack are the quark-line attachments G_1..G_k
 *                (G_1 pushed first, nearest the antiquark): out = ubar (i g gamma.G_k) S ...
 *                S (i g gamma.G_1) v, S(q) = i (qslash + m)/(q^2 - m^2); colour factor
 *                (t^{a_k} .. t^{a_1})_{ij} stripped.  Must be the last op.
 * Each current carries its summed incoming momentum.  Returns 0, or -1 on a malformed
 * program. */
int or_tree_amp(int proc, const double *params, const double *p, int h, const int *prog, int len,
                double *out)
{
    if (!is_qcd(proc) || proc == P_GG_GG) return -1;
    tables();
    real par[3];
    load_par(params, par);
    ext_t X;
    setup_qcd(proc, p, par, h, 0, &X);
    real g = X.g;
    cplx J[16][4];
    real P[16][4];
    int sp = 0;
    for (int t = 0; t < len; ++t) {
        int op = prog[t];
        if (op >= 0) {
            if (op >= X.ng || sp >= 16) return -1;
            memcpy(J[sp], X.e[op], sizeof J[sp]);
            memcpy(P[sp], X.q[op], sizeof P[sp]);
            ++sp;
        } else if (op == -1) {
            if (sp < 2) return -1;
            cplx V[4];
            real Q[4];
            vvv(J[sp - 2], P[sp - 2], J[sp - 1], P[sp - 1], V);
            for (int mu = 0; mu < 4; ++mu) Q[mu] = P[sp - 2][mu] + P[sp - 1][mu];
            cplx f = -I / dot_rr(Q, Q);
            sp -= 2;
            for (int mu = 0; mu < 4; ++mu) {
                J[sp][mu] = f * g * V[mu];
                P[sp][mu] = Q[mu];
            }
            ++sp;
        } else if (op >= -4) {
            if (sp < 3) return -1;
            int s = -2 - op;
            const cplx *A = J[sp - 3], *B = J[sp - 2], *C = J[sp - 1];
            cplx ab = dot_cc(A, B), ac = dot_cc(A, C), bc = dot_cc(B, C), L[4];
            real Q[4];
            for (int mu = 0; mu < 4; ++mu) {
                if (s == 0) L[mu] = B[mu] * ac - C[mu] * ab;
                else if (s == 1) L[mu] = A[mu] * bc - C[mu] * ab;
                else L[mu] = A[mu] * bc - B[mu] * ac;
                Q[mu] = P[sp - 3][mu] + P[sp - 2][mu] + P[sp - 1][mu];
            }
            cplx f = -I / dot_rr(Q, Q);
            sp -= 3;
            for (int mu = 0; mu < 4; ++mu) {
                J[sp][mu] = f * (-I * g * g) * L[mu];
                P[sp][mu] = Q[mu];
            }
            ++sp;
        } else {
            int k = -10 - op;
            if (k < 1 || k != sp || t != len - 1) return -1;
            cplx psi[4], tmp[4];
            memcpy(psi, X.v, sizeof psi);
            real q[4];
            for (int mu = 0; mu < 4; ++mu) q[mu] = -X.pa[mu];
            for (int a = 0; a < k; ++a) {
                vertex_q(J[a], g, psi, tmp);
                if (a == k - 1) {
                    cplx r = rowcol(X.ubar, tmp);
                    out[0] = (double)creal(r);
                    out[1] = (double)cimag(r);
                    return 0;
                }
                for (int mu = 0; mu < 4; ++mu) q[mu] += P[a][mu];
                prop_q(q, X.m, tmp, psi);
            }
        }
    }
    return -1;
}

/* Brute force: averaged sum over all helicities and ALL explicit colour assignments of
 * |M|^2 from the colour-dressed recursion (no colour matrix, no decomposition). */
double or_me_brute_colour(int proc, const double *params, const double *p)
{
    if (!is_qcd(proc)) return -1;
    tables();
    real par[3];
    load_par(params, par);
    int n_par = N_PAR[proc];
    int nh = 1 << n_par;
    real sum = 0;
    dressed_t *D = malloc(sizeof(dressed_t));
    for (int h = 0; h < nh; ++h) {
        ext_t X;
        setup_qcd(proc, p, par, h, 0, &X);
        int n = X.ng;
        if (proc == P_GG_GG) {
            int amp_set = (1 << (n - 1)) - 1;
            int ncol = 1 << (3 * (n - 1));
            for (int cc = 0; cc < ncol; ++cc) {
                int col[NG_MAX];
                for (int i = 0, x = cc; i < n - 1; ++i, x /= 8) col[i] = x % 8;
                dressed_currents(&X, n - 1, col, amp_set, D);
                for (int a = 0; a < 8; ++a) {
                    cplx m = dot_cc(D->J[amp_set][a], X.e[n - 1]);
                    sum += creal(m * conj(m));
                }
            }
        } else {
            int ncol = 1 << (3 * n);
            for (int cc = 0; cc < ncol; ++cc) {
                int col[NG_MAX];
                for (int i = 0, x = cc; i < n; ++i, x /= 8) col[i] = x % 8;
                dressed_currents(&X, n, col, 0, D);
                for (int j = 0; j < 3; ++j) {
                    cplx out[3];
                    dressed_qline(&X, D, j, out);
                    for (int i = 0; i < 3; ++i) sum += creal(out[i] * conj(out[i]));
                }
            }
        }
    }
    free(D);
    return (double)(sum / 256);
}

/* external-state completeness checks: sum_lam u ubar, sum_lam v vbar (4x4, re/im
 * interleaved, row-major) and sum_lam eps^mu eps^nu* (4x4) for momentum p, mass m */
int or_spin_sums(const double *p, double m, int basis, double *uu, double *vv, double *ee)
{
    tables();
    real pr[4] = {p[0], p[1], p[2], p[3]};
    cplx U[4][4], V[4][4], E[4][4];
    memset(U, 0, sizeof U); memset(V, 0, sizeof V); memset(E, 0, sizeof E);
    for (int lam = -1; lam <= 1; lam += 2) {
        cplx u[4], ub[4], v[4], vb[4], e[4];
        if (basis == 1 && m > 0) { spinor_z(pr, m, lam, 0, u); spinor_z(pr, m, lam, 1, v); }
        else { spinor_u(pr, m, lam, u); spinor_v(pr, m, lam, v); }
        dirac_bar(u, ub);
        dirac_bar(v, vb);
        polvec(pr, lam, 0, basis, e);
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) {
                U[i][j] += u[i] * ub[j];
                V[i][j] += v[i] * vb[j];
                E[i][j] += e[i] * conj(e[j]);
            }
    }
    for (int i = 0; i < 16; ++i) {
        uu[2 * i] = (double)creal(U[i / 4][i % 4]); uu[2 * i + 1] = (double)cimag(U[i / 4][i % 4]);
        vv[2 * i] = (double)creal(V[i / 4][i % 4]); vv[2 * i + 1] = (double)cimag(V[i / 4][i % 4]);
        ee[2 * i] = (double)creal(E[i / 4][i % 4]); ee[2 * i + 1] = (double)cimag(E[i / 4][i % 4]);
    }
    return 0;
}

/* the Dirac matrices, for the Clifford-algebra check: out[mu][i][j] re/im interleaved */
int or_gamma(double *out)
{
    tables();
    for (int mu = 0; mu < 4; ++mu)
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) {
                out[2 * ((mu * 4 + i) * 4 + j)] = (double)creal(GAM[mu][i][j]);
                out[2 * ((mu * 4 + i) * 4 + j) + 1] = (double)cimag(GAM[mu][i][j]);
            }
    return 0;
}

/* f^{abc} as computed from the Gell-Mann matrices */
int or_fabc(double *out)
{
    tables();
    for (int i = 0; i < 512; ++i) out[i] = (double)(&FABC[0][0][0])[i];
    return 0;
}
