/*
 * Direct Wick-contraction oracle for baryon-baryon four-point correlators.
 *
 * TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the CPU
 * baseline of the benchmark; never by the product path.
 *
 * Computes, for the requested relative coordinates r, the plain definition
 *
 *   C(r)_{a b a' b'} = sum_X sum_{terms} w1 w2 w3 w4
 *       sum_{xi, xi'} T1(xi_1 xi_2 xi_3; a) T2(xi_4 xi_5 xi_6; b)
 *                     T3(xi'_1 xi'_2 xi'_3; a') T4(xi'_4 xi'_5 xi'_6; b')
 *       < q_1 .. q_6  qbar'_6 .. qbar'_1 >
 *
 * with q_1..q_3 the fields of B1 at X+r (periodic), q_4..q_6 those of B2 at X
 * (Sec. 3, Eq. (LN.pLLp.ududsu) and its coordinate assignment), and the source
 * antiquarks in the mirrored order written there.  For that order Wick's theorem
 * gives the determinant of the 6x6 propagator matrix
 *     P_ij = [f_i == f'_j] S_{f_i}(x_i)[xi_i][xi'_j]
 * (Sec. 3, Eq. (Qexchdiag)), i.e. a signed sum over flavour-preserving
 * bijections sigma of sink fields onto source fields.
 *
 * T(xi_a xi_b xi_c; g) = eps(c_a c_b c_c) Gamma_1(mu_a, mu_b) Gamma_2(g, mu_c), per
 * baryon, from the general interpolating field of Sec. 2, Eq. (FieldOperator_B)
 * (the octet fields of Sec. 2 have Gamma_1 = C gamma_5 and Gamma_2 = 1); xi = 3*mu + c.
 * The source tensor is the sink tensor with primed indices, exactly as printed
 * in Sec. 3.
 *
 * Evaluation order (plain, no FFT): the sum over the sink indices xi of one
 * baryon is done first at each site, giving
 *     G(x; g; e_a, e_b, e_c) = sum_xi T(xi; g) S_fa(x)[xi_a][e_a] S_fb(x)[xi_b][e_b] S_fc(x)[xi_c][e_c]
 * and then, for each sigma and each nonzero source-tensor entry, the product
 * G1(X+r; a; e'_{sigma(1..3)}) G2(X; b; e'_{sigma(4..6)}) is summed over X.
 * The cost is O(V^2) per channel and time slice.
 */
#include <complex.h>
#include <stdlib.h>
#include <string.h>

typedef double _Complex cplx;

#define NE 1728 /* 12^3 */

static int perm_sign(const int *p, int n) {
    int q[8], s = 1;
    for (int i = 0; i < n; ++i) q[i] = p[i];
    for (int i = 0; i < n; ++i)
        while (q[i] != i) { int j = q[i]; int t = q[j]; q[j] = j; q[i] = t; s = -s; }
    return s;
}

static double eps3(int a, int b, int c) {
    if (a == b || b == c || a == c) return 0.0;
    if ((a == 0 && b == 1) || (a == 1 && b == 2) || (a == 2 && b == 0)) return 1.0;
    return -1.0;
}

/* Nonzero entries of one baryon tensor T(e_a e_b e_c; g). */
typedef struct { int e[3]; cplx v; } nzent;

#define MAXNZ 384 /* 6 colour orders x 16 Gamma_1 entries x 4 Gamma_2 entries */

static int tensor_nz(const cplx *M1, const cplx *M2, int g, nzent *out) {
    int n = 0;
    for (int ca = 0; ca < 3; ++ca) for (int cb = 0; cb < 3; ++cb) for (int cc = 0; cc < 3; ++cc) {
        double e = eps3(ca, cb, cc);
        if (e == 0.0) continue;
        for (int ma = 0; ma < 4; ++ma) for (int mb = 0; mb < 4; ++mb) for (int mc = 0; mc < 4; ++mc) {
            cplx m = M1[4 * ma + mb] * M2[4 * g + mc];
            if (m == 0) continue;
            out[n].e[0] = 3 * ma + ca; out[n].e[1] = 3 * mb + cb; out[n].e[2] = 3 * mc + cc;
            out[n].v = e * m;
            ++n;
        }
    }
    return n;
}

static const cplx *prop(const cplx *Sl, const cplx *Ss, int f, long x) {
    return (f == 2 ? Ss : Sl) + x * 144;
}

/* G(x; g; .) for one sink term, for g in {g_lo, g_lo+1}, all sites. */
static void build_G(long V, const cplx *Sl, const cplx *Ss, const nzent *nz, const int *nnz,
                    const int *f, cplx *G) {   /* nz: [2][MAXNZ], the entries for g_lo and g_lo+1 */
#pragma omp parallel for schedule(static)
    for (long x = 0; x < V; ++x) {
        const cplx *Sa = prop(Sl, Ss, f[0], x), *Sb = prop(Sl, Ss, f[1], x), *Sc = prop(Sl, Ss, f[2], x);
        for (int g = 0; g < 2; ++g) {
            cplx *Gx = G + (x * 2 + g) * NE;
            memset(Gx, 0, sizeof(cplx) * NE);
            for (int k = 0; k < nnz[g]; ++k) {
                const nzent *t = &nz[g * MAXNZ + k];
                const cplx *ra = Sa + 12 * t->e[0], *rb = Sb + 12 * t->e[1], *rc = Sc + 12 * t->e[2];
                for (int ea = 0; ea < 12; ++ea) {
                    cplx va = t->v * ra[ea];
                    for (int eb = 0; eb < 12; ++eb) {
                        cplx vab = va * rb[eb];
                        cplx *dst = Gx + 144 * ea + 12 * eb;
                        for (int ec = 0; ec < 12; ++ec) dst[ec] += vab * rc[ec];
                    }
                }
            }
        }
    }
}

/* One entry of the flattened work list: a (sigma, source-tensor entry pair) with
   its sign and weight, the G-index of each sink baryon, and the source spins. */
typedef struct { int t1, t2; int A, B; int sp; cplx coef; } work;

/*
 * Arguments
 *   Lx,Ly,Lz     lattice extent; sites ordered x fastest, then y, then z.
 *   Sl, Ss       light / strange propagator of one time slice, [V][12][12] complex (re,im).
 *   M1, M2       per baryon B1..B4, the 4x4 complex matrices Gamma_1 and Gamma_2,
 *                [4][4][4] row-major (octet fields: C gamma_5 and the identity).
 *   nterm[4]     number of terms of B1, B2, B3, B4 (at most 3 each).
 *   w[4][3]      term weights.
 *   flav[4][3][3] flavour of each field of each term (0 = u, 1 = d, 2 = s), field order a,b,c.
 *   glo[4]       per baryon B1..B4, the first of its two spin components computed
 *                (0: the upper two, 2: the lower two; Sec. 6 uses the upper two of
 *                every baryon forward in time and the lower two backward).
 *   nr, r[nr][3] relative coordinates.
 *   out[nr][16]  complex result, spin index a + 2*(b + 2*(a' + 2*b')), each spin
 *                relative to its baryon's glo.
 * Returns 0, or a negative value on bad input or allocation failure.
 */
int oracle_wick(int Lx, int Ly, int Lz, const double *Sl_, const double *Ss_, const double *M1_,
                const double *M2_, const int *nterm, const double *w, const int *flav, const int *glo,
                int nr, const int *r, double *out_) {
    const cplx *Sl = (const cplx *)Sl_, *Ss = (const cplx *)Ss_;
    const cplx *M1 = (const cplx *)M1_, *M2 = (const cplx *)M2_;
    cplx *out = (cplx *)out_;
    long V = (long)Lx * Ly * Lz;
    for (int b = 0; b < 4; ++b) if (nterm[b] < 1 || nterm[b] > 3) return -1;
    for (int b = 0; b < 4; ++b) if (glo[b] != 0 && glo[b] != 2) return -1;

    /* tensor nonzeros of every baryon for its two spin components g = glo[b], glo[b]+1 */
    nzent *nz = malloc(sizeof(nzent) * 4 * 2 * MAXNZ);
    int nnz[4][2];
    if (!nz) return -3;
    for (int b = 0; b < 4; ++b)
        for (int g = 0; g < 2; ++g) nnz[b][g] = tensor_nz(M1 + 16 * b, M2 + 16 * b, glo[b] + g, nz + (2 * b + g) * MAXNZ);

    /* G tensors of every sink term of B1 and B2 */
    int n1 = nterm[0], n2 = nterm[1];
    cplx *G1 = malloc(sizeof(cplx) * (size_t)n1 * V * 2 * NE);
    cplx *G2 = malloc(sizeof(cplx) * (size_t)n2 * V * 2 * NE);
    if (!G1 || !G2) { free(G1); free(G2); free(nz); return -3; }
    for (int t = 0; t < n1; ++t)
        build_G(V, Sl, Ss, nz, nnz[0], flav + (0 * 3 + t) * 3, G1 + (size_t)t * V * 2 * NE);
    for (int t = 0; t < n2; ++t)
        build_G(V, Sl, Ss, nz + 2 * MAXNZ, nnz[1], flav + (1 * 3 + t) * 3, G2 + (size_t)t * V * 2 * NE);
    const nzent *nz3 = nz + 4 * MAXNZ, *nz4 = nz + 6 * MAXNZ;

    /* flattened work list over term tuples, sigma and source nonzeros */
    size_t cap = 1024, nw = 0;
    work *wl = malloc(sizeof(work) * cap);
    if (!wl) { free(G1); free(G2); free(nz); return -3; }
    for (int t1 = 0; t1 < nterm[0]; ++t1) for (int t2 = 0; t2 < nterm[1]; ++t2)
    for (int t3 = 0; t3 < nterm[2]; ++t3) for (int t4 = 0; t4 < nterm[3]; ++t4) {
        int fs[6], fsrc[6];
        for (int i = 0; i < 3; ++i) {
            fs[i] = flav[(0 * 3 + t1) * 3 + i]; fs[3 + i] = flav[(1 * 3 + t2) * 3 + i];
            fsrc[i] = flav[(2 * 3 + t3) * 3 + i]; fsrc[3 + i] = flav[(3 * 3 + t4) * 3 + i];
        }
        double wt = w[0 * 3 + t1] * w[1 * 3 + t2] * w[2 * 3 + t3] * w[3 * 3 + t4];
        /* all permutations of 6 (Heap-free: lexicographic enumeration) */
        int p[6] = {0, 1, 2, 3, 4, 5};
        for (;;) {
            int ok = 1;
            for (int i = 0; i < 6; ++i) if (fs[i] != fsrc[p[i]]) { ok = 0; break; }
            if (ok) {
                int sg = perm_sign(p, 6);
                for (int a3 = 0; a3 < 2; ++a3) for (int a4 = 0; a4 < 2; ++a4)
                for (int k3 = 0; k3 < nnz[2][a3]; ++k3) for (int k4 = 0; k4 < nnz[3][a4]; ++k4) {
                    const nzent *n3 = &nz3[MAXNZ * a3 + k3], *n4 = &nz4[MAXNZ * a4 + k4];
                    int e[6];
                    for (int i = 0; i < 3; ++i) { e[i] = n3->e[i]; e[3 + i] = n4->e[i]; }
                    if (nw == cap) {
                        cap *= 2;
                        work *nwl = realloc(wl, sizeof(work) * cap);
                        if (!nwl) { free(wl); free(G1); free(G2); free(nz); return -3; }
                        wl = nwl;
                    }
                    work *q = &wl[nw++];
                    q->t1 = t1; q->t2 = t2;
                    q->A = 144 * e[p[0]] + 12 * e[p[1]] + e[p[2]];
                    q->B = 144 * e[p[3]] + 12 * e[p[4]] + e[p[5]];
                    q->sp = a3 + 2 * a4;
                    q->coef = wt * sg * n3->v * n4->v;
                }
            }
            /* next permutation */
            int i = 4;
            while (i >= 0 && p[i] > p[i + 1]) --i;
            if (i < 0) break;
            int j = 5;
            while (p[j] < p[i]) --j;
            int t = p[i]; p[i] = p[j]; p[j] = t;
            for (int a = i + 1, b = 5; a < b; ++a, --b) { t = p[a]; p[a] = p[b]; p[b] = t; }
        }
    }

    /* direct O(V^2) sum over X.  Summation: double partial sums over chunks of
       the work list, flushed into long double accumulators per (r, X block).  The
       sum has ~V * |work| terms of random sign; plain recursive double summation
       loses ~sqrt(N) eps (about 1e-12 relative at 16^3), this keeps the oracle's
       own rounding near 1e-15.  Work is shared over (r, X block) pairs. */
    const long XB = 64;
    const long nxb = (V + XB - 1) / XB;
    long double _Complex *tot = calloc((size_t)nr * 16, sizeof(long double _Complex));
    if (!tot) { free(wl); free(G1); free(G2); free(nz); return -3; }
#pragma omp parallel
    {
        long double _Complex *acc = calloc((size_t)nr * 16, sizeof(long double _Complex));
#pragma omp for schedule(dynamic, 1)
        for (long job = 0; job < (long)nr * nxb; ++job) {
            if (!acc) continue;
            int ir = (int)(job / nxb);
            long X0 = (job % nxb) * XB, X1 = X0 + XB < V ? X0 + XB : V;
            int rx = r[3 * ir], ry = r[3 * ir + 1], rz = r[3 * ir + 2];
            for (long X = X0; X < X1; ++X) {
                int x = (int)(X % Lx), y = (int)((X / Lx) % Ly), z = (int)(X / ((long)Lx * Ly));
                long x1 = (long)(((x + rx) % Lx + Lx) % Lx) + (long)Lx * ((((y + ry) % Ly + Ly) % Ly)
                          + (long)Ly * (((z + rz) % Lz + Lz) % Lz));
                for (size_t k0 = 0; k0 < nw; k0 += 1024) {
                    size_t k1 = k0 + 1024 < nw ? k0 + 1024 : nw;
                    cplx part[16];
                    for (int s = 0; s < 16; ++s) part[s] = 0;
                    for (size_t k = k0; k < k1; ++k) {
                        const work *q = &wl[k];
                        const cplx *g1 = G1 + ((size_t)q->t1 * V + x1) * 2 * NE + q->A;
                        const cplx *g2 = G2 + ((size_t)q->t2 * V + X) * 2 * NE + q->B;
                        cplx u0 = q->coef * g1[0], u1 = q->coef * g1[NE];
                        cplx v0 = g2[0], v1 = g2[NE];
                        cplx *o = part + 4 * q->sp;
                        o[0] += u0 * v0; o[1] += u1 * v0; o[2] += u0 * v1; o[3] += u1 * v1;
                    }
                    for (int s = 0; s < 16; ++s) acc[(size_t)ir * 16 + s] += part[s];
                }
            }
        }
#pragma omp critical
        {
            if (acc)
                for (size_t i = 0; i < (size_t)nr * 16; ++i) tot[i] += acc[i];
        }
        free(acc);
    }
    for (size_t i = 0; i < (size_t)nr * 16; ++i) out[i] = (cplx)tot[i];
    free(tot);
    free(wl); free(G1); free(G2); free(nz);
    return 0;
}
