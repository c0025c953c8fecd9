/*
 * qvm_oracle.c -- plain FP64 CPU oracle for the full-amplitude state-vector
 * method (Schroedinger simulation: every gate is a linear map on all 2^n
 * amplitudes; paper, "Multi-simulation methods", noise-free simulation).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or constant
 * with the HIP library; gate matrices are derived here from their
 * definitions, independently.
 *
 * Conventions (the paper is silent on all of them; readings listed in the
 * design notes):
 *   - qubit q <-> bit q of the amplitude index (qubit 0 = least significant);
 *   - amplitudes stored interleaved (re, im) in double precision;
 *   - a k-qubit gate matrix is row-major 2^k x 2^k complex, and bit r of its
 *     row/column index refers to targets[r];
 *   - controls are 1-controls given as a bit mask over qubits.
 *
 * Reductions use Neumaier-compensated FP64 summation over a fixed chunking
 * that does not depend on the thread count, so results are deterministic.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <stddef.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXK 6

/* ------------------------------------------------------------------ */
/* Compensated summation (Neumaier's variant of Kahan summation).      */
/* ------------------------------------------------------------------ */
typedef struct { double s, c; } orc_acc;

static inline void acc_add(orc_acc* a, double x) {
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else                       a->c += (x - t) + a->s;
    a->s = t;
}
static inline double acc_get(const orc_acc* a) { return a->s + a->c; }

#define ORC_NCHUNK 256

int orc_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count of the parallel loops that follow (timing legs only). */
void orc_set_threads(int t) {
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/* ------------------------------------------------------------------ */
/* Gate matrices.  The paper names the gates (H, X, Y, Z, S, T, RX, RY, */
/* RZ, U3, CNOT, CZ, CR, Toffoli, arbitrary unitaries) but prints no    */
/* matrices; these are the textbook definitions.                        */
/* Returns the number of target qubits k, or -1 for an unknown name.    */
/* u receives 2^k x 2^k complex entries, row-major, (re, im) pairs.     */
/* ------------------------------------------------------------------ */
static void set_c(double* u, int dim, int r, int c, double re, double im) {
    u[2 * (r * dim + c)] = re;
    u[2 * (r * dim + c) + 1] = im;
}

int orc_gate_matrix(const char* name, const double* p, double* u) {
    const double s2 = 1.0 / sqrt(2.0);
    int k = 1;
    if (!strcmp(name, "rzz") || !strcmp(name, "swap")) k = 2;
    int dim = 1 << k;
    memset(u, 0, sizeof(double) * 2 * dim * dim);
    if (!strcmp(name, "i")) {
        set_c(u, 2, 0, 0, 1, 0); set_c(u, 2, 1, 1, 1, 0);
    } else if (!strcmp(name, "h")) {
        set_c(u, 2, 0, 0, s2, 0); set_c(u, 2, 0, 1, s2, 0);
        set_c(u, 2, 1, 0, s2, 0); set_c(u, 2, 1, 1, -s2, 0);
    } else if (!strcmp(name, "x")) {
        set_c(u, 2, 0, 1, 1, 0); set_c(u, 2, 1, 0, 1, 0);
    } else if (!strcmp(name, "y")) {
        set_c(u, 2, 0, 1, 0, -1); set_c(u, 2, 1, 0, 0, 1);
    } else if (!strcmp(name, "z")) {
        set_c(u, 2, 0, 0, 1, 0); set_c(u, 2, 1, 1, -1, 0);
    } else if (!strcmp(name, "s")) {
        set_c(u, 2, 0, 0, 1, 0); set_c(u, 2, 1, 1, 0, 1);
    } else if (!strcmp(name, "sdg")) {
        set_c(u, 2, 0, 0, 1, 0); set_c(u, 2, 1, 1, 0, -1);
    } else if (!strcmp(name, "t")) {
        set_c(u, 2, 0, 0, 1, 0); set_c(u, 2, 1, 1, cos(M_PI / 4), sin(M_PI / 4));
    } else if (!strcmp(name, "tdg")) {
        set_c(u, 2, 0, 0, 1, 0); set_c(u, 2, 1, 1, cos(M_PI / 4), -sin(M_PI / 4));
    } else if (!strcmp(name, "rx")) {
        /* exp(-i theta X / 2) = cos(theta/2) I - i sin(theta/2) X */
        double c = cos(p[0] / 2), s = sin(p[0] / 2);
        set_c(u, 2, 0, 0, c, 0); set_c(u, 2, 0, 1, 0, -s);
        set_c(u, 2, 1, 0, 0, -s); set_c(u, 2, 1, 1, c, 0);
    } else if (!strcmp(name, "ry")) {
        /* exp(-i theta Y / 2) = cos(theta/2) I - i sin(theta/2) Y */
        double c = cos(p[0] / 2), s = sin(p[0] / 2);
        set_c(u, 2, 0, 0, c, 0); set_c(u, 2, 0, 1, -s, 0);
        set_c(u, 2, 1, 0, s, 0); set_c(u, 2, 1, 1, c, 0);
    } else if (!strcmp(name, "rz")) {
        /* exp(-i theta Z / 2) = diag(e^{-i theta/2}, e^{+i theta/2}) */
        double h = p[0] / 2;
        set_c(u, 2, 0, 0, cos(h), -sin(h)); set_c(u, 2, 1, 1, cos(h), sin(h));
    } else if (!strcmp(name, "p")) {
        /* phase gate diag(1, e^{i theta}); with one control this is CR */
        set_c(u, 2, 0, 0, 1, 0); set_c(u, 2, 1, 1, cos(p[0]), sin(p[0]));
    } else if (!strcmp(name, "u3")) {
        /* U3(theta, phi, lambda) in the OpenQASM 2 form */
        double c = cos(p[0] / 2), s = sin(p[0] / 2);
        double ph = p[1], la = p[2];
        set_c(u, 2, 0, 0, c, 0);
        set_c(u, 2, 0, 1, -cos(la) * s, -sin(la) * s);
        set_c(u, 2, 1, 0, cos(ph) * s, sin(ph) * s);
        set_c(u, 2, 1, 1, cos(ph + la) * c, sin(ph + la) * c);
    } else if (!strcmp(name, "rzz")) {
        /* exp(-i theta Z(x)Z / 2): phase e^{-i theta/2} where the two bits
           agree, e^{+i theta/2} where they differ */
        double h = p[0] / 2;
        for (int j = 0; j < 4; ++j) {
            int parity = (j & 1) ^ ((j >> 1) & 1);
            set_c(u, 4, j, j, cos(h), parity ? sin(h) : -sin(h));
        }
    } else if (!strcmp(name, "swap")) {
        set_c(u, 4, 0, 0, 1, 0); set_c(u, 4, 1, 2, 1, 0);
        set_c(u, 4, 2, 1, 1, 0); set_c(u, 4, 3, 3, 1, 0);
    } else {
        return -1;
    }
    return k;
}

/* ------------------------------------------------------------------ */
/* State initialisation: basis state |x>.                               */
/* ------------------------------------------------------------------ */
void orc_init_basis(double* psi, int n, uint64_t x) {
    uint64_t N = (uint64_t)1 << n;
    memset(psi, 0, sizeof(double) * 2 * N);
    psi[2 * x] = 1.0;
}

/* ------------------------------------------------------------------ */
/* Gate application by definition: for every index b whose target bits */
/* are 0 and whose control bits are all 1, gather the 2^k amplitudes    */
/* b + sum_r j_r 2^{t_r}, multiply by U, scatter back.                  */
/* ------------------------------------------------------------------ */
void orc_apply(double* psi, int n, const double* u, int k, const int* t,
               uint64_t cmask) {
    uint64_t N = (uint64_t)1 << n;
    int dim = 1 << k;
    uint64_t tmask = 0;
    for (int r = 0; r < k; ++r) tmask |= (uint64_t)1 << t[r];
    int64_t NN = (int64_t)N;
#pragma omp parallel for schedule(static) if (NN >= (1 << 14))
    for (int64_t bb = 0; bb < NN; ++bb) {
        uint64_t b = (uint64_t)bb;
        if (b & tmask) continue;
        if ((b & cmask) != cmask) continue;
        uint64_t idx[1 << ORC_MAXK];
        double vr[1 << ORC_MAXK], vi[1 << ORC_MAXK];
        for (int j = 0; j < dim; ++j) {
            uint64_t off = 0;
            for (int r = 0; r < k; ++r)
                if ((j >> r) & 1) off |= (uint64_t)1 << t[r];
            idx[j] = b | off;
            vr[j] = psi[2 * idx[j]];
            vi[j] = psi[2 * idx[j] + 1];
        }
        for (int i = 0; i < dim; ++i) {
            double ar = 0, ai = 0;
            for (int j = 0; j < dim; ++j) {
                double mr = u[2 * (i * dim + j)], mi = u[2 * (i * dim + j) + 1];
                ar += mr * vr[j] - mi * vi[j];
                ai += mr * vi[j] + mi * vr[j];
            }
            psi[2 * idx[i]] = ar;
            psi[2 * idx[i] + 1] = ai;
        }
    }
}

/* Apply a whole gate list (matrices concatenated in mats, offsets in
   doubles given by mat_off; targets 6 per gate). */
void orc_run(double* psi, int n, int64_t ngates, const double* mats,
             const int64_t* mat_off, const int* ks, const int* targets,
             const uint64_t* cmasks) {
    for (int64_t g = 0; g < ngates; ++g)
        orc_apply(psi, n, mats + mat_off[g], ks[g], targets + 6 * g, cmasks[g]);
}

/* ------------------------------------------------------------------ */
/* Probabilities p_i = |psi_i|^2 (paper, "A variety of convenient tools":
   quantum state, probability and expectation readout).                 */
/* ------------------------------------------------------------------ */
void orc_probabilities(const double* psi, int n, double* p) {
    int64_t N = (int64_t)1 << n;
#pragma omp parallel for schedule(static) if (N >= (1 << 14))
    for (int64_t i = 0; i < N; ++i)
        p[i] = psi[2 * i] * psi[2 * i] + psi[2 * i + 1] * psi[2 * i + 1];
}

/* Marginal over qubits q[0..m-1]: out[j] = sum of p_i over i whose bits at
   q equal j (bit r of j <-> q[r]).  Sequential compensated sums. */
void orc_marginal(const double* psi, int n, int m, const int* q, double* out) {
    uint64_t N = (uint64_t)1 << n, M = (uint64_t)1 << m;
    orc_acc* acc = (orc_acc*)calloc(M, sizeof(orc_acc));
    for (uint64_t i = 0; i < N; ++i) {
        uint64_t j = 0;
        for (int r = 0; r < m; ++r) j |= ((i >> q[r]) & 1) << r;
        acc_add(&acc[j], psi[2 * i] * psi[2 * i] + psi[2 * i + 1] * psi[2 * i + 1]);
    }
    for (uint64_t j = 0; j < M; ++j) out[j] = acc_get(&acc[j]);
    free(acc);
}

/* Squared norm sum_i |psi_i|^2 (chunked compensated sum). */
double orc_norm2(const double* psi, int n) {
    int64_t N = (int64_t)1 << n;
    double part[ORC_NCHUNK];
#pragma omp parallel for schedule(static) if (N >= (1 << 14))
    for (int c = 0; c < ORC_NCHUNK; ++c) {
        int64_t lo = N * c / ORC_NCHUNK, hi = N * (c + 1) / ORC_NCHUNK;
        orc_acc a = {0, 0};
        for (int64_t i = lo; i < hi; ++i)
            acc_add(&a, psi[2 * i] * psi[2 * i] + psi[2 * i + 1] * psi[2 * i + 1]);
        part[c] = acc_get(&a);
    }
    orc_acc t = {0, 0};
    for (int c = 0; c < ORC_NCHUNK; ++c) acc_add(&t, part[c]);
    return acc_get(&t);
}

static inline int popc64(uint64_t v) { return __builtin_popcountll(v); }

/* ------------------------------------------------------------------ */
/* Pauli-string expectation in symplectic form: X-part mask x, Z-part   */
/* mask z (a Y sets both).  With P = i^{|x&z|} X^x Z^z,                 */
/*   <psi|P|psi> = sum_i conj(psi_{i^x}) i^{|x&z|} (-1)^{|z&i|} psi_i.  */
/* Returns the real part; *im_out receives the imaginary part, which is */
/* zero up to rounding for a Hermitian P.                               */
/* ------------------------------------------------------------------ */
double orc_expect_pauli(const double* psi, int n, uint64_t x, uint64_t z,
                        double* im_out) {
    int64_t N = (int64_t)1 << n;
    double pre[ORC_NCHUNK], pim[ORC_NCHUNK];
#pragma omp parallel for schedule(static) if (N >= (1 << 14))
    for (int c = 0; c < ORC_NCHUNK; ++c) {
        int64_t lo = N * c / ORC_NCHUNK, hi = N * (c + 1) / ORC_NCHUNK;
        orc_acc ar = {0, 0}, ai = {0, 0};
        for (int64_t i = lo; i < hi; ++i) {
            uint64_t j = (uint64_t)i ^ x;
            double a_r = psi[2 * j], a_i = -psi[2 * j + 1];   /* conj(psi_j) */
            double b_r = psi[2 * i], b_i = psi[2 * i + 1];
            double pr = a_r * b_r - a_i * b_i, pi = a_r * b_i + a_i * b_r;
            if (popc64(z & (uint64_t)i) & 1) { pr = -pr; pi = -pi; }
            acc_add(&ar, pr);
            acc_add(&ai, pi);
        }
        pre[c] = acc_get(&ar);
        pim[c] = acc_get(&ai);
    }
    orc_acc tr = {0, 0}, ti = {0, 0};
    for (int c = 0; c < ORC_NCHUNK; ++c) { acc_add(&tr, pre[c]); acc_add(&ti, pim[c]); }
    double sr = acc_get(&tr), si = acc_get(&ti);
    /* multiply by i^{|x&z|} */
    double rr = sr, ri = si;
    switch (popc64(x & z) & 3) {
        case 1: rr = -si; ri = sr; break;
        case 2: rr = -sr; ri = -si; break;
        case 3: rr = si; ri = -sr; break;
        default: break;
    }
    if (im_out) *im_out = ri;
    return rr;
}

/* out = P psi for one Pauli string: (P psi)_i = i^{|x&z|} (-1)^{|z&(i^x)|}
   psi_{i^x}.  out and psi must not alias. */
void orc_apply_pauli(const double* psi, int n, uint64_t x, uint64_t z,
                     double coeff, double* out, int accumulate) {
    int64_t N = (int64_t)1 << n;
    int c = popc64(x & z) & 3;
#pragma omp parallel for schedule(static) if (N >= (1 << 14))
    for (int64_t i = 0; i < N; ++i) {
        uint64_t j = (uint64_t)i ^ x;
        double vr = psi[2 * j], vi = psi[2 * j + 1];
        if (popc64(z & j) & 1) { vr = -vr; vi = -vi; }
        double wr = vr, wi = vi;
        switch (c) {
            case 1: wr = -vi; wi = vr; break;
            case 2: wr = -vr; wi = -vi; break;
            case 3: wr = vi; wi = -vr; break;
            default: break;
        }
        if (accumulate) { out[2 * i] += coeff * wr; out[2 * i + 1] += coeff * wi; }
        else            { out[2 * i] = coeff * wr;  out[2 * i + 1] = coeff * wi; }
    }
}

/* ------------------------------------------------------------------ */
/* Sampling (paper: Measure / directly_run).  C_i = sum_{j<=i} p_j in   */
/* index order (compensated); the sample for uniform u is the smallest  */
/* i with C_i > u * C_{N-1}.  margin[s] receives the distance of the    */
/* scaled target to the nearer CDF boundary of the chosen bin, so that  */
/* a caller can tell samples that sit on a boundary.                    */
/* ------------------------------------------------------------------ */
typedef struct { double u; int64_t s; } orc_us;
static int cmp_us(const void* a, const void* b) {
    double x = ((const orc_us*)a)->u, y = ((const orc_us*)b)->u;
    return (x > y) - (x < y);
}

void orc_sample(const double* psi, int n, int64_t ns, const double* uni,
                uint64_t* out, double* margin) {
    uint64_t N = (uint64_t)1 << n;
    double total = orc_norm2(psi, n);
    orc_us* ord = (orc_us*)malloc(sizeof(orc_us) * (size_t)(ns > 0 ? ns : 1));
    for (int64_t s = 0; s < ns; ++s) { ord[s].u = uni[s]; ord[s].s = s; }
    qsort(ord, (size_t)ns, sizeof(orc_us), cmp_us);
    orc_acc c = {0, 0};
    double prev = 0.0;
    uint64_t i = 0;
    double ci = 0.0;
    int have = 0;
    for (int64_t q = 0; q < ns; ++q) {
        double target = ord[q].u * total;
        for (;;) {
            if (!have) {
                prev = acc_get(&c);
                acc_add(&c, psi[2 * i] * psi[2 * i] + psi[2 * i + 1] * psi[2 * i + 1]);
                ci = acc_get(&c);
                have = 1;
            }
            if (ci > target || i == N - 1) break;
            ++i;
            have = 0;
        }
        out[ord[q].s] = i;
        if (margin) {
            double m1 = fabs(target - prev), m2 = fabs(ci - target);
            margin[ord[q].s] = m1 < m2 ? m1 : m2;
        }
    }
    free(ord);
}

/* ------------------------------------------------------------------ */
/* Adjoint gradient of f(theta) = <psi(theta)|H|psi(theta)> with        */
/* H = sum_k c_k P_k, for circuits whose parameterised gates are        */
/* U_l = exp(-i theta_l G_l / 2), G_l a Pauli on the gate's target.     */
/* Published reverse-sweep method (Jones & Gacon, arXiv:2009.02823):    */
/*   psi_L = U_L..U_1|0>, lambda_L = H psi_L;                           */
/*   for l = L..1: if U_l has a parameter,                              */
/*       df/dtheta_l = Im <lambda_l| G_l |psi_l>;                       */
/*     then psi <- U_l^dagger psi, lambda <- U_l^dagger lambda.         */
/* gen[g] = 0 for a fixed gate, 1/2/3 for generator X/Y/Z; pidx[g] is   */
/* the parameter index.  The forward circuit starts from |0..0>.        */
/* ------------------------------------------------------------------ */
static void dagger(const double* u, int k, double* ud) {
    int dim = 1 << k;
    for (int i = 0; i < dim; ++i)
        for (int j = 0; j < dim; ++j) {
            ud[2 * (i * dim + j)] = u[2 * (j * dim + i)];
            ud[2 * (i * dim + j) + 1] = -u[2 * (j * dim + i) + 1];
        }
}

static double inner_im(const double* a, const double* b, int n) {
    /* Im sum conj(a_i) b_i, chunked compensated */
    int64_t N = (int64_t)1 << n;
    double part[ORC_NCHUNK];
#pragma omp parallel for schedule(static) if (N >= (1 << 14))
    for (int c = 0; c < ORC_NCHUNK; ++c) {
        int64_t lo = N * c / ORC_NCHUNK, hi = N * (c + 1) / ORC_NCHUNK;
        orc_acc s = {0, 0};
        for (int64_t i = lo; i < hi; ++i)
            acc_add(&s, a[2 * i] * b[2 * i + 1] - a[2 * i + 1] * b[2 * i]);
        part[c] = acc_get(&s);
    }
    orc_acc t = {0, 0};
    for (int c = 0; c < ORC_NCHUNK; ++c) acc_add(&t, part[c]);
    return acc_get(&t);
}

static double inner_re(const double* a, const double* b, int n) {
    int64_t N = (int64_t)1 << n;
    double part[ORC_NCHUNK];
#pragma omp parallel for schedule(static) if (N >= (1 << 14))
    for (int c = 0; c < ORC_NCHUNK; ++c) {
        int64_t lo = N * c / ORC_NCHUNK, hi = N * (c + 1) / ORC_NCHUNK;
        orc_acc s = {0, 0};
        for (int64_t i = lo; i < hi; ++i)
            acc_add(&s, a[2 * i] * b[2 * i] + a[2 * i + 1] * b[2 * i + 1]);
        part[c] = acc_get(&s);
    }
    orc_acc t = {0, 0};
    for (int c = 0; c < ORC_NCHUNK; ++c) acc_add(&t, part[c]);
    return acc_get(&t);
}

int orc_adjoint(int n, int64_t ngates, const double* mats, const int64_t* mat_off,
                const int* ks, const int* targets, const uint64_t* cmasks,
                const int* gen, const int* pidx, int64_t nterms,
                const uint64_t* xs, const uint64_t* zs, const double* cs,
                double* f_out, double* grad) {
    uint64_t N = (uint64_t)1 << n;
    double* psi = (double*)malloc(sizeof(double) * 2 * N);
    double* lam = (double*)calloc(2 * N, sizeof(double));
    double* tmp = (double*)malloc(sizeof(double) * 2 * N);
    if (!psi || !lam || !tmp) { free(psi); free(lam); free(tmp); return -1; }
    orc_init_basis(psi, n, 0);
    orc_run(psi, n, ngates, mats, mat_off, ks, targets, cmasks);
    for (int64_t k = 0; k < nterms; ++k)
        orc_apply_pauli(psi, n, xs[k], zs[k], cs[k], lam, 1);
    *f_out = inner_re(psi, lam, n);
    double ud[2 * 64 * 64];
    for (int64_t g = ngates - 1; g >= 0; --g) {
        int kk = ks[g];
        const int* t = targets + 6 * g;
        if (gen[g]) {
            uint64_t gx = 0, gz = 0, bit = (uint64_t)1 << t[0];
            if (gen[g] == 1) gx = bit;
            else if (gen[g] == 2) { gx = bit; gz = bit; }
            else gz = bit;
            /* tmp = G psi restricted to the control subspace: a controlled
               rotation's generator acts only where the controls are 1. */
            orc_apply_pauli(psi, n, gx, gz, 1.0, tmp, 0);
            if (cmasks[g]) {
                int64_t NN = (int64_t)N;
                for (int64_t i = 0; i < NN; ++i)
                    if (((uint64_t)i & cmasks[g]) != cmasks[g]) { tmp[2 * i] = 0; tmp[2 * i + 1] = 0; }
            }
            grad[pidx[g]] += inner_im(lam, tmp, n);
        }
        dagger(mats + mat_off[g], kk, ud);
        orc_apply(psi, n, ud, kk, t, cmasks[g]);
        orc_apply(lam, n, ud, kk, t, cmasks[g]);
    }
    free(psi); free(lam); free(tmp);
    return 0;
}
