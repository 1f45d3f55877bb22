/*
 * CPU oracle for state-vector simulation of quantum circuits.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the GPU library includes, links or
 * calls this file; only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg load it. It shares no code, header or table with the GPU
 * path.
 *
 * Plain complex128 arithmetic, one gate at a time, in place, exactly as the
 * paper defines the operations (Haener & Steiger, "0.5 Petabyte Simulation of
 * a 45-Qubit Quantum Circuit", Sec. 2 and Sec. 3.2):
 *   - amplitude index i = sum_q b_q 2^q, qubit q is bit q (Sec. 2, the X_0
 *     example on two qubits);
 *   - a single-qubit gate U on qubit q multiplies the state by
 *     1 x ... x U x 1 x ... x 1 with q identities to its right (Sec. 2);
 *   - a k-qubit gate gathers, for every assignment c of the n-k other bits,
 *     the 2^k amplitudes whose target bits spell x (bit j of x at qubit
 *     qubits[j]), multiplies by the 2^k x 2^k matrix and scatters the result
 *     back (Sec. 3.2);
 *   - the named gate matrices are the ones printed in Sec. 2.
 * Built with -O2 -ffp-contract=off (no fused multiply-add), no fast-math.
 * The only parallelism is an OpenMP split of independent index ranges.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------ gate matrices */
/* 2x2 complex, row-major, (re, im) interleaved: m[(2*r + c)*2 + {0,1}]. */
static void gate_matrix(const char* name, double m[8]) {
    const double s = 1.0 / sqrt(2.0);
    const double c4 = cos(M_PI / 4.0), s4 = sin(M_PI / 4.0);
    memset(m, 0, 8 * sizeof(double));
#define SET(r, c, re, im) do { m[((r) * 2 + (c)) * 2] = (re); m[((r) * 2 + (c)) * 2 + 1] = (im); } while (0)
    if (!strcmp(name, "H")) {          /* H = (1/sqrt2) [[1, 1], [1, -1]] */
        SET(0, 0, s, 0); SET(0, 1, s, 0); SET(1, 0, s, 0); SET(1, 1, -s, 0);
    } else if (!strcmp(name, "T")) {   /* T = diag(1, e^{i pi/4}) */
        SET(0, 0, 1, 0); SET(1, 1, c4, s4);
    } else if (!strcmp(name, "TDG")) { /* T^dagger = diag(1, e^{-i pi/4}) */
        SET(0, 0, 1, 0); SET(1, 1, c4, -s4);
    } else if (!strcmp(name, "SX")) {  /* X^1/2 = 1/2 [[1+i, 1-i], [1-i, 1+i]] */
        SET(0, 0, 0.5, 0.5); SET(0, 1, 0.5, -0.5); SET(1, 0, 0.5, -0.5); SET(1, 1, 0.5, 0.5);
    } else if (!strcmp(name, "SXDG")) {/* conjugate transpose of X^1/2 */
        SET(0, 0, 0.5, -0.5); SET(0, 1, 0.5, 0.5); SET(1, 0, 0.5, 0.5); SET(1, 1, 0.5, -0.5);
    } else if (!strcmp(name, "SY")) {  /* Y^1/2 = 1/2 [[1+i, -1-i], [1+i, 1+i]] */
        SET(0, 0, 0.5, 0.5); SET(0, 1, -0.5, -0.5); SET(1, 0, 0.5, 0.5); SET(1, 1, 0.5, 0.5);
    } else if (!strcmp(name, "SYDG")) {/* conjugate transpose of Y^1/2 */
        SET(0, 0, 0.5, -0.5); SET(0, 1, 0.5, -0.5); SET(1, 0, -0.5, 0.5); SET(1, 1, 0.5, -0.5);
    } else if (!strcmp(name, "X")) {   /* X = [[0, 1], [1, 0]] */
        SET(0, 1, 1, 0); SET(1, 0, 1, 0);
    } else if (!strcmp(name, "Y")) {   /* Y = [[0, -i], [i, 0]] */
        SET(0, 1, 0, -1); SET(1, 0, 0, 1);
    } else if (!strcmp(name, "Z")) {   /* Z = diag(1, -1) */
        SET(0, 0, 1, 0); SET(1, 1, -1, 0);
    } else {
        m[0] = NAN;
    }
#undef SET
}

int oracle_gate_matrix(const char* name, double* out8) {
    gate_matrix(name, out8);
    return isnan(out8[0]) ? -1 : 0;
}

/* ------------------------------------------------------------ gate application */
/* Single-qubit gate U on qubit q: pairs (i, i | 2^q) with bit q of i clear. */
void oracle_apply_1q(double* psi, int n, int q, const double* u) {
    const int64_t half = (int64_t)1 << (n - 1);
    const int64_t low = ((int64_t)1 << q) - 1;
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < half; ++p) {
        const int64_t i = ((p & ~low) << 1) | (p & low);
        const int64_t j = i | ((int64_t)1 << q);
        const double ar = psi[2 * i], ai = psi[2 * i + 1];
        const double br = psi[2 * j], bi = psi[2 * j + 1];
        /* new_i = u00 a + u01 b ; new_j = u10 a + u11 b */
        const double n0r = (u[0] * ar - u[1] * ai) + (u[2] * br - u[3] * bi);
        const double n0i = (u[0] * ai + u[1] * ar) + (u[2] * bi + u[3] * br);
        const double n1r = (u[4] * ar - u[5] * ai) + (u[6] * br - u[7] * bi);
        const double n1i = (u[4] * ai + u[5] * ar) + (u[6] * bi + u[7] * br);
        psi[2 * i] = n0r; psi[2 * i + 1] = n0i;
        psi[2 * j] = n1r; psi[2 * j + 1] = n1i;
    }
}

/* CZ on qubits a, b: multiply by -1 every amplitude whose bits a and b are 1
 * (CZ = diag(1, 1, 1, -1), Sec. 2). */
void oracle_apply_cz(double* psi, int n, int a, int b) {
    const int64_t dim = (int64_t)1 << n;
    const int64_t m = ((int64_t)1 << a) | ((int64_t)1 << b);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < dim; ++i) {
        if ((i & m) == m) {
            psi[2 * i] = -psi[2 * i];
            psi[2 * i + 1] = -psi[2 * i + 1];
        }
    }
}

/* Dense k-qubit gate (Sec. 3.2). qubits[j] is the state bit carrying bit j of
 * the matrix row/column index; u is 2^k x 2^k complex, row-major, (re, im)
 * interleaved. For every c, v[x] = psi[c + dep(x)] and
 * psi[c + dep(y)] = sum_x u[y][x] v[x]. */
int oracle_apply_dense(double* psi, int n, int k, const int* qubits, const double* u) {
    if (k < 1 || k > n || k > 12) return -1;
    int64_t tmask = 0;
    for (int j = 0; j < k; ++j) {
        if (qubits[j] < 0 || qubits[j] >= n) return -1;
        if (tmask & ((int64_t)1 << qubits[j])) return -1;
        tmask |= (int64_t)1 << qubits[j];
    }
    const int d = 1 << k;
    const int64_t nc = (int64_t)1 << (n - k);
    int64_t* off = (int64_t*)malloc(sizeof(int64_t) * d);
    for (int x = 0; x < d; ++x) {
        int64_t o = 0;
        for (int j = 0; j < k; ++j)
            if ((x >> j) & 1) o |= (int64_t)1 << qubits[j];
        off[x] = o;
    }
#pragma omp parallel
    {
        double* v = (double*)malloc(sizeof(double) * 2 * d);
#pragma omp for schedule(static)
        for (int64_t c = 0; c < nc; ++c) {
            /* deposit the bits of c, in order, into the non-target positions */
            int64_t base = 0, rest = c;
            for (int bit = 0, used = 0; bit < n && used < n - k; ++bit) {
                if (tmask & ((int64_t)1 << bit)) continue;
                if (rest & 1) base |= (int64_t)1 << bit;
                rest >>= 1;
                ++used;
            }
            for (int x = 0; x < d; ++x) {
                v[2 * x] = psi[2 * (base | off[x])];
                v[2 * x + 1] = psi[2 * (base | off[x]) + 1];
            }
            for (int y = 0; y < d; ++y) {
                double sr = 0.0, si = 0.0;
                for (int x = 0; x < d; ++x) {
                    const double mr = u[2 * (y * d + x)], mi = u[2 * (y * d + x) + 1];
                    sr += mr * v[2 * x] - mi * v[2 * x + 1];
                    si += mr * v[2 * x + 1] + mi * v[2 * x];
                }
                psi[2 * (base | off[y])] = sr;
                psi[2 * (base | off[y]) + 1] = si;
            }
        }
        free(v);
    }
    free(off);
    return 0;
}

/* Apply a named gate (or CZ). Returns -1 for an unknown name. */
int oracle_apply_named(double* psi, int n, const char* name, int q0, int q1) {
    if (!strcmp(name, "CZ")) {
        if (q0 < 0 || q0 >= n || q1 < 0 || q1 >= n || q0 == q1) return -1;
        oracle_apply_cz(psi, n, q0, q1);
        return 0;
    }
    double u[8];
    gate_matrix(name, u);
    if (isnan(u[0]) || q0 < 0 || q0 >= n) return -1;
    oracle_apply_1q(psi, n, q0, u);
    return 0;
}

/* ------------------------------------------------------------ circuit text */
/* Circuit text: "n <qubits>" then one gate per line: "<NAME> q0 [q1]" or
 * "U k q0 .. q(k-1) re im re im ..." (2 * 4^k numbers, row-major). */
static const char* skip_ws(const char* p) {
    while (*p == ' ' || *p == '\t' || *p == '\r') ++p;
    return p;
}

/* Apply every gate of the circuit text to psi (whose 2^n amplitudes the
 * caller initialised). Returns the number of gates applied, or -(line) on a
 * parse error. */
long oracle_apply_text(double* psi, int n, const char* text) {
    const char* p = text;
    long line = 0, applied = 0;
    int nfile = -1;
    while (*p) {
        ++line;
        const char* eol = strchr(p, '\n');
        if (!eol) eol = p + strlen(p);
        p = skip_ws(p);
        if (p < eol && *p != '#') {
            char name[16] = {0};
            int len = 0;
            while (p < eol && *p != ' ' && *p != '\t' && len < 15) name[len++] = *p++;
            if (!strcmp(name, "n")) {
                nfile = (int)strtol(p, NULL, 10);
                if (nfile != n) return -line;
            } else if (!strcmp(name, "U")) {
                char* e;
                int k = (int)strtol(p, &e, 10);
                p = e;
                if (k < 1 || k > 12) return -line;
                int qs[12];
                for (int j = 0; j < k; ++j) { qs[j] = (int)strtol(p, &e, 10); if (e == p) return -line; p = e; }
                const int cnt = 2 << (2 * k);
                double* u = (double*)malloc(sizeof(double) * cnt);
                for (int t = 0; t < cnt; ++t) { u[t] = strtod(p, &e); if (e == p) { free(u); return -line; } p = e; }
                int rc = oracle_apply_dense(psi, n, k, qs, u);
                free(u);
                if (rc) return -line;
                ++applied;
            } else {
                char* e;
                int q0 = (int)strtol(p, &e, 10);
                if (e == p) return -line;
                p = e;
                int q1 = -1;
                if (!strcmp(name, "CZ")) { q1 = (int)strtol(p, &e, 10); if (e == p) return -line; }
                if (oracle_apply_named(psi, n, name, q0, q1)) return -line;
                ++applied;
            }
        }
        p = (*eol) ? eol + 1 : eol;
    }
    return applied;
}

/* |0...0> then every gate of the text. */
long oracle_run_text(double* psi, int n, const char* text) {
    const int64_t dim = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < 2 * dim; ++i) psi[i] = 0.0;
    psi[0] = 1.0;
    return oracle_apply_text(psi, n, text);
}

/* ------------------------------------------------------------ cluster matrix */
/* The 2^k x 2^k matrix of a gate sequence acting on k qubits: column x is the
 * result of applying the gates, in order, to basis vector e_x of the k-qubit
 * space (qubit positions inside the text are 0..k-1). */
long oracle_cluster_matrix(int k, const char* text, double* out) {
    const int d = 1 << k;
    double* col = (double*)malloc(sizeof(double) * 2 * d);
    for (int x = 0; x < d; ++x) {
        memset(col, 0, sizeof(double) * 2 * d);
        col[2 * x] = 1.0;
        long rc = oracle_apply_text(col, k, text);
        if (rc < 0) { free(col); return rc; }
        for (int y = 0; y < d; ++y) {
            out[2 * (y * d + x)] = col[2 * y];
            out[2 * (y * d + x) + 1] = col[2 * y + 1];
        }
    }
    free(col);
    return 0;
}

/* ------------------------------------------------------------ reductions */
/* norm = sum |a_i|^2, sum_p2 = sum p_i^2, entropy = -sum p_i ln p_i with
 * p_i = |a_i|^2 (0 ln 0 = 0). Accumulated in long double. */
void oracle_stats(const double* psi, int n, double* norm, double* sum_p2, double* entropy) {
    const int64_t dim = (int64_t)1 << n;
    long double s1 = 0.0L, s2 = 0.0L, se = 0.0L;
#pragma omp parallel for schedule(static) reduction(+ : s1, s2, se)
    for (int64_t i = 0; i < dim; ++i) {
        const double p = psi[2 * i] * psi[2 * i] + psi[2 * i + 1] * psi[2 * i + 1];
        s1 += p;
        s2 += (long double)p * p;
        if (p > 0.0) se -= (long double)p * log(p);
    }
    *norm = (double)s1;
    *sum_p2 = (double)s2;
    *entropy = (double)se;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
