/* Sanitizer driver for the CPU oracle (built with -fsanitize=address,undefined
 * by tests/test_sanitizers_cpu.py): random circuits as text, dense gates of
 * every size, malformed input, the cluster matrix and the reductions. Exits
 * non-zero when a result is inconsistent; the sanitizers report memory errors
 * and undefined behaviour themselves. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

long oracle_run_text(double* psi, int n, const char* text);
long oracle_apply_text(double* psi, int n, const char* text);
int oracle_apply_dense(double* psi, int n, int k, const int* qubits, const double* u);
long oracle_cluster_matrix(int k, const char* text, double* out);
void oracle_stats(const double* psi, int n, double* norm, double* sum_p2, double* entropy);
int oracle_gate_matrix(const char* name, double* out8);

static uint64_t rng_state = 0x1234567ull;
static uint64_t next_u64(void) { /* xorshift64* */
    rng_state ^= rng_state >> 12;
    rng_state ^= rng_state << 25;
    rng_state ^= rng_state >> 27;
    return rng_state * 2685821657736338717ull;
}
static int below(int m) { return (int)(next_u64() % (uint64_t)m); }

static void append(char** buf, size_t* len, size_t* cap, const char* s) {
    size_t l = strlen(s);
    if (*len + l + 1 > *cap) {
        *cap = 2 * (*len + l + 1);
        *buf = (char*)realloc(*buf, *cap);
    }
    memcpy(*buf + *len, s, l + 1);
    *len += l;
}

/* A random circuit over n qubits: named gates, CZs and dense k-qubit gates
 * with the identity matrix (so the norm stays exactly 1). */
static char* random_circuit(int n, int gates) {
    static const char* names[] = {"H", "T", "SX", "SY", "X", "Y", "Z", "TDG", "SXDG", "SYDG"};
    size_t len = 0, cap = 256;
    char* buf = (char*)malloc(cap);
    buf[0] = 0;
    char line[64];
    snprintf(line, sizeof line, "n %d\n", n);
    append(&buf, &len, &cap, line);
    for (int g = 0; g < gates; ++g) {
        int kind = below(10);
        if (kind < 6 || n < 2) {
            snprintf(line, sizeof line, "%s %d\n", names[below(10)], below(n));
            append(&buf, &len, &cap, line);
        } else if (kind < 9) {
            int a = below(n), b = below(n - 1);
            if (b >= a) ++b;
            snprintf(line, sizeof line, "CZ %d %d\n", a, b);
            append(&buf, &len, &cap, line);
        } else {
            int k = 1 + below(n < 4 ? n : 4);
            int used[32] = {0}, qs[4];
            for (int j = 0; j < k; ++j) {
                int q;
                do q = below(n); while (used[q]);
                used[q] = 1;
                qs[j] = q;
            }
            snprintf(line, sizeof line, "U %d", k);
            append(&buf, &len, &cap, line);
            for (int j = 0; j < k; ++j) {
                snprintf(line, sizeof line, " %d", qs[j]);
                append(&buf, &len, &cap, line);
            }
            int d = 1 << k;
            for (int r = 0; r < d; ++r)
                for (int c = 0; c < d; ++c) append(&buf, &len, &cap, r == c ? " 1 0" : " 0 0");
            append(&buf, &len, &cap, "\n");
        }
    }
    return buf;
}

int main(void) {
    int bad = 0;
    for (int trial = 0; trial < 60; ++trial) {
        int n = 1 + below(12);
        char* text = random_circuit(n, 5 + below(60));
        double* psi = (double*)malloc(sizeof(double) * 2 * ((size_t)1 << n));
        long rc = oracle_run_text(psi, n, text);
        double norm, s2, ent;
        oracle_stats(psi, n, &norm, &s2, &ent);
        if (rc < 0 || fabs(norm - 1.0) > 1e-12) {
            fprintf(stderr, "trial %d: rc %ld norm %.17g\n", trial, rc, norm);
            bad = 1;
        }
        free(psi);
        free(text);
    }
    /* cluster matrix of a short sequence on k qubits */
    for (int k = 1; k <= 6; ++k) {
        char* text = random_circuit(k, 20);
        double* m = (double*)malloc(sizeof(double) * 2 * ((size_t)1 << (2 * k)));
        if (oracle_cluster_matrix(k, text, m) < 0) bad = 1;
        free(m);
        free(text);
    }
    /* malformed input is reported as a parse error, not read past */
    const char* broken[] = {"n 3\nH\n", "n 3\nCZ 1\n", "n 3\nU 2 0\n", "n 3\nU 1 0 1 0 0\n",
                            "n 3\nQQQQQQQQQQQQQQQQQQQQQQQQ 1\n", "n 4\nH 0\n", "n 3\nH 7\n", "n 3\nU 13 0 1\n"};
    double psi3[16];
    for (size_t i = 0; i < sizeof broken / sizeof broken[0]; ++i)
        if (oracle_run_text(psi3, 3, broken[i]) >= 0) {
            fprintf(stderr, "malformed input %zu accepted\n", i);
            bad = 1;
        }
    double g[8];
    if (oracle_gate_matrix("H", g) != 0 || oracle_gate_matrix("NOPE", g) == 0) bad = 1;
    printf("oracle driver done: %s\n", bad ? "FAILED" : "ok");
    return bad;
}
