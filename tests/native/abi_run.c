/* abi_run.c -- drive libptqmc through its C ABI alone (no Python, no torch): read one
 * instance from a text file, run n_cycles PT cycles with a library-owned workspace and
 * stream, and print the observables and spins as text.
 *
 *   abi_run <instance.txt> <seed> <sweeps_per_exchange> <n_cycles> [encoding [flags]]
 *
 * instance.txt: "N M R n_edges n_colors", then n_edges lines "i j J", then N values of h,
 * N colours, R values of b, R values of K (whitespace separated; b and K as %a hex
 * floats so they round-trip exactly).  Output lines: "E_cl ...", "C ...", "rung_of ...",
 * "replica_of ...", "acc ...", "att ...", "roundtrips ...", "label ...", "sumE ...",
 * "sumC ...", "sumE2 ...", "sumC2 ...", "nup ...", "ndown ...", "counters t e n_acc",
 * "spins ..." (R x M x N values in {-1, +1} by slot, slice, site) and, with
 * PT_FLAG_TAU_CORR among the flags, "sumCt ..." (R x PT_TAU_LAGS by rung).  Exit status 0
 * on success, 1 on a library error (its message on stderr). */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "ptqmc.h"

static int check(int rc, const char *what)
{
    if (rc != PT_OK) {
        fprintf(stderr, "%s: %s (%s)\n", what, pt_strerror(rc), pt_last_error());
        return 1;
    }
    return 0;
}

static void put_i64(const char *name, const int64_t *v, int n)
{
    printf("%s", name);
    for (int i = 0; i < n; ++i) printf(" %lld", (long long)v[i]);
    printf("\n");
}

static void put_u64(const char *name, const uint64_t *v, int n)
{
    printf("%s", name);
    for (int i = 0; i < n; ++i) printf(" %llu", (unsigned long long)v[i]);
    printf("\n");
}

static void put_i32(const char *name, const int32_t *v, int n)
{
    printf("%s", name);
    for (int i = 0; i < n; ++i) printf(" %d", (int)v[i]);
    printf("\n");
}

int main(int argc, char **argv)
{
    if (argc < 5 || argc > 7) {
        fprintf(stderr, "usage: %s instance.txt seed sweeps_per_exchange n_cycles [encoding [flags]]\n",
                argv[0]);
        return 2;
    }
    const int encoding = argc > 5 ? atoi(argv[5]) : PT_INT8;
    const uint32_t flags = argc > 6 ? (uint32_t)strtoul(argv[6], NULL, 0) : 0u;
    FILE *f = fopen(argv[1], "r");
    if (!f) {
        perror(argv[1]);
        return 2;
    }
    int N, M, R, E, ncol;
    if (fscanf(f, "%d %d %d %d %d", &N, &M, &R, &E, &ncol) != 5) return 2;
    int32_t *ei = calloc(E > 0 ? E : 1, 4), *ej = calloc(E > 0 ? E : 1, 4);
    int8_t *J = calloc(E > 0 ? E : 1, 1), *h = calloc(N, 1);
    uint8_t *col = calloc(N, 1);
    double *b = calloc(R, 8), *K = calloc(R, 8);
    for (int e = 0; e < E; ++e) {
        int a, c, w;
        if (fscanf(f, "%d %d %d", &a, &c, &w) != 3) return 2;
        ei[e] = a;
        ej[e] = c;
        J[e] = (int8_t)w;
    }
    for (int i = 0; i < N; ++i) {
        int v;
        if (fscanf(f, "%d", &v) != 1) return 2;
        h[i] = (int8_t)v;
    }
    for (int i = 0; i < N; ++i) {
        int v;
        if (fscanf(f, "%d", &v) != 1) return 2;
        col[i] = (uint8_t)v;
    }
    for (int r = 0; r < R; ++r)
        if (fscanf(f, "%la", &b[r]) != 1) return 2;
    for (int r = 0; r < R; ++r)
        if (fscanf(f, "%la", &K[r]) != 1) return 2;
    fclose(f);

    const pt_instance inst = {N, M, R, E, ncol, ei, ej, J, h, col, b, K};
    const pt_options opt = {strtoull(argv[2], NULL, 0), atoi(argv[3]), encoding, flags, 0, 0, 0};
    pt_ctx *ctx = NULL;
    if (check(pt_init(&ctx, &inst, 1, &opt, NULL, NULL, 0), "pt_init")) return 1;
    if (check(pt_run(ctx, atoi(argv[4])), "pt_run")) return 1;

    int64_t *E_cl = calloc(R, 8), *C = calloc(R, 8), *sE = calloc(R, 8), *sC = calloc(R, 8),
            *sE2 = calloc(R, 8), *sC2 = calloc(R, 8);
    int32_t *rung_of = calloc(R, 4), *replica_of = calloc(R, 4);
    uint64_t *acc = calloc(R, 8), *att = calloc(R, 8), *rt = calloc(R, 8), *nup = calloc(R, 8),
             *ndown = calloc(R, 8);
    int8_t *label = calloc(R, 1), *spins = calloc((size_t)R * M * N, 1);
    int64_t *sCt = calloc((size_t)R * PT_TAU_LAGS, 8);
    pt_obs o = {E_cl, C, rung_of, replica_of, acc, att, rt, label, sE, sC, sE2, sC2, nup, ndown,
                0, 0, 0, sCt};
    if (check(pt_observables(ctx, 0, &o), "pt_observables")) return 1;
    if (check(pt_get_spins(ctx, 0, spins), "pt_get_spins")) return 1;
    put_i64("E_cl", E_cl, R);
    put_i64("C", C, R);
    put_i32("rung_of", rung_of, R);
    put_i32("replica_of", replica_of, R);
    put_u64("acc", acc, R - 1);
    put_u64("att", att, R - 1);
    put_u64("roundtrips", rt, R);
    printf("label");
    for (int c = 0; c < R; ++c) printf(" %d", (int)label[c]);
    printf("\n");
    put_i64("sumE", sE, R);
    put_i64("sumC", sC, R);
    put_i64("sumE2", sE2, R);
    put_i64("sumC2", sC2, R);
    put_u64("nup", nup, R);
    put_u64("ndown", ndown, R);
    printf("counters %llu %llu %llu\n", (unsigned long long)o.t, (unsigned long long)o.e,
           (unsigned long long)o.n_acc);
    printf("spins");
    for (size_t k = 0; k < (size_t)R * M * N; ++k) printf(" %d", (int)spins[k]);
    printf("\n");
    if (flags & PT_FLAG_TAU_CORR) put_i64("sumCt", sCt, R * PT_TAU_LAGS);
    pt_free(ctx);
    return 0;
}
