/*
 * Test support: runs the oracle from a descriptor file, so that the oracle can be built with
 * AddressSanitizer and UndefinedBehaviorSanitizer as a program of its own (a sanitized shared
 * library loaded into Python would need its runtime preloaded).
 *
 *   oracle_sanitize_runner <descriptor file> <result file>
 *
 * Descriptor file (written by tests/test_oracle_sanitizers.py, host byte order):
 *   int64 sizeof(ko_desc); the bytes of a ko_desc whose pointers are rewritten here; then one
 *   array per pointer of the descriptor, in the order read_arrays() takes them, each as int64
 *   element count (0: NULL) followed by the elements (8-byte doubles, 4-byte ints for planes);
 *   then int64 pid_begin, pid_end, digests flag, history flag.
 * Result file: the tallies in the order of ko_tallies, each array whole (digests and history
 * only when asked for, the energy-resolved times only when the descriptor has energy bins).
 * Exit status 0 on success, 2 for a malformed file, 3 when ko_run reports an error.
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "karl_oracle.h"

static FILE* in;

static int rd(void* p, size_t n) { return fread(p, 1, n, in) == n; }

/* one array: its element count, then the elements; NULL for a count of 0 */
static void* rd_array(size_t elem, int64_t* count_out) {
    int64_t n = 0;
    if (!rd(&n, sizeof n) || n < 0) exit(2);
    if (count_out) *count_out = n;
    if (n == 0) return NULL;
    void* p = malloc((size_t)n * elem);
    if (!p || !rd(p, (size_t)n * elem)) exit(2);
    return p;
}

static void read_arrays(ko_desc* d) {
    d->n_gas = rd_array(8, NULL);
    for (int s = 0; s < KO_MAX_SPECIES; ++s) d->n_field[s] = rd_array(8, NULL);
    for (int s = 0; s < KO_MAX_SPECIES; ++s) {
        d->sp[s].edges = rd_array(8, NULL);
        d->sp[s].dens_edges = rd_array(8, NULL);
    }
    for (int i = 0; i < KO_MAX_PROC; ++i) {
        d->proc[i].xs = rd_array(8, NULL);
        d->proc[i].ang_edges = rd_array(8, NULL);
        d->proc[i].ang_theta = rd_array(8, NULL);
        d->proc[i].ang_pdf = rd_array(8, NULL);
    }
    d->planes = rd_array(4, NULL);
    d->e_field = rd_array(8, NULL);
    d->b_field = rd_array(8, NULL);
}

static void wr(FILE* f, const void* p, size_t n) {
    if (n && fwrite(p, 1, n, f) != n) exit(2);
}

int main(int argc, char** argv) {
    if (argc != 3) {
        fprintf(stderr, "usage: %s <descriptor file> <result file>\n", argv[0]);
        return 2;
    }
    in = fopen(argv[1], "rb");
    if (!in) return 2;
    int64_t size = 0;
    if (!rd(&size, sizeof size) || size != (int64_t)sizeof(ko_desc)) {
        fprintf(stderr, "descriptor of %lld bytes, this build's has %zu\n", (long long)size, sizeof(ko_desc));
        return 2;
    }
    ko_desc d;
    if (!rd(&d, sizeof d)) return 2;
    read_arrays(&d);
    int64_t run[4];
    if (!rd(run, sizeof run)) return 2;
    fclose(in);

    const size_t ns = (size_t)(d.n_species ? d.n_species : 2);
    const size_t nr = (size_t)d.n_r, nz = (size_t)d.n_z, nb = (size_t)d.n_bins;
    const size_t np = (size_t)d.n_planes, nd = (size_t)d.n_dens_bins;
    const size_t n_dt = ns * nr * nz, n_jz = ns * nr * (nz + 1) * 2, n_jr = ns * (nr + 1) * nz * 2;
    const size_t n_sp = ns * np * 2 * (nb + 2), n_e = nd ? ns * nr * nz * (nd + 2) : 0;
    const size_t n_dig = run[2] ? (size_t)d.n_primaries : 0, n_hist = run[3] ? (size_t)d.n_primaries * KO_NHIST : 0;
    ko_tallies t;
    memset(&t, 0, sizeof t);
    t.counters = calloc(KO_NCOUNTERS, 8);
    t.ledger = calloc(KO_NLEDGER, 8);
    t.density_time = calloc(n_dt, 8);
    t.recomb = calloc(n_dt, 8);
    t.jz = calloc(n_jz, 8);
    t.jr = calloc(n_jr, 8);
    t.spectra = calloc(n_sp, 8);
    t.digests = n_dig ? calloc(n_dig, 8) : NULL;
    t.hist = n_hist ? calloc(n_hist, 8) : NULL;
    t.density_time_e = n_e ? calloc(n_e, 8) : NULL;
    const int rc = ko_run(&d, run[0], run[1], &t);
    if (rc != 0) {
        fprintf(stderr, "ko_run returned %d\n", rc);
        return 3;
    }
    FILE* out = fopen(argv[2], "wb");
    if (!out) return 2;
    wr(out, t.counters, 8 * KO_NCOUNTERS);
    wr(out, t.ledger, 8 * KO_NLEDGER);
    wr(out, t.density_time, 8 * n_dt);
    wr(out, t.recomb, 8 * n_dt);
    wr(out, t.jz, 8 * n_jz);
    wr(out, t.jr, 8 * n_jr);
    wr(out, t.spectra, 8 * n_sp);
    wr(out, t.digests, 8 * n_dig);
    wr(out, t.hist, 8 * n_hist);
    wr(out, t.density_time_e, 8 * n_e);
    fclose(out);

    free(t.counters); free(t.ledger); free(t.density_time); free(t.recomb); free(t.jz);
    free(t.jr); free(t.spectra); free(t.digests); free(t.hist); free(t.density_time_e);
    free((void*)d.n_gas);
    for (int s = 0; s < KO_MAX_SPECIES; ++s) {
        free((void*)d.n_field[s]);
        free((void*)d.sp[s].edges);
        free((void*)d.sp[s].dens_edges);
    }
    for (int i = 0; i < KO_MAX_PROC; ++i) {
        free((void*)d.proc[i].xs);
        free((void*)d.proc[i].ang_edges);
        free((void*)d.proc[i].ang_theta);
        free((void*)d.proc[i].ang_pdf);
    }
    free((void*)d.planes); free((void*)d.e_field); free((void*)d.b_field);
    return 0;
}
