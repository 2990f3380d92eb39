/* The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer: a
 * small network read from raw arrays (dir/name.bin, written by the test) is
 * simulated in both precision modes, replayed from its own raster, and freed.
 * The oracle is included as source so that the whole of it is instrumented. */
#include <stdio.h>
#include <stdlib.h>

#include "../../oracle/hines_oracle.c"

static void *load(const char *dir, const char *name, long *count, long elem)
{
    char path[1024];
    snprintf(path, sizeof path, "%s/%s.bin", dir, name);
    FILE *f = fopen(path, "rb");
    if (!f) { fprintf(stderr, "missing %s\n", path); exit(2); }
    fseek(f, 0, SEEK_END);
    long bytes = ftell(f);
    fseek(f, 0, SEEK_SET);
    void *p = malloc(bytes > 0 ? bytes : 1);
    if (bytes > 0 && fread(p, 1, bytes, f) != (size_t)bytes) exit(2);
    fclose(f);
    *count = bytes / elem;
    return p;
}

int main(int argc, char **argv)
{
    if (argc < 3) return 2;
    const char *dir = argv[1];
    const int64_t steps = atoll(argv[2]);
    long n_off, nc, nn, ns;
    int64_t *off = load(dir, "comp_off", &n_off, 8);
    int32_t *parent = load(dir, "parent", &nc, 4);
    double *len = load(dir, "length_um", &nc, 8);
    double *diam = load(dir, "diam_um", &nc, 8);
    uint8_t *mech = load(dir, "mech", &nc, 1);
    int32_t *det = load(dir, "detector", &nn, 4);
    double *iext = load(dir, "iext_nA", &nn, 8);
    int32_t *pre = load(dir, "syn_pre", &ns, 4);
    int32_t *post = load(dir, "syn_post", &ns, 4);
    int32_t *comp = load(dir, "syn_comp", &ns, 4);
    int32_t *delay = load(dir, "syn_delay", &ns, 4);
    double *w = load(dir, "syn_w", &ns, 8);
    const int32_t N = (int32_t)(n_off - 1);
    long total = 0;
    for (int prec = 0; prec <= 1; ++prec) {
        orc_params_t P = {0.025, 0.5, 2.0, 0.0, 0.0, -65.0, 1.0, 100.0, 0.12, 0.036, 0.0003,
                          50.0, -77.0, -54.3, 1e-4, -65.0, prec};
        orc_sim_t *o = orc_create(&P, N, off, parent, len, diam, mech, det, iext, ns, pre, post,
                                  comp, delay, w, steps);
        if (!o || orc_step(o, steps) != 0) return 1;
        const int64_t nspk = orc_n_spikes(o);
        int64_t *spk = malloc(sizeof(int64_t) * 2 * (nspk > 0 ? nspk : 1));
        orc_get_spikes(o, spk);
        /* replay the run's own raster into a second simulation */
        uint8_t *raster = calloc((size_t)(steps + 1) * N, 1);
        for (int64_t k = 0; k < nspk; ++k) raster[spk[2 * k + 1] * N + spk[2 * k]] = 1;
        orc_sim_t *r = orc_create(&P, N, off, parent, len, diam, mech, det, iext, ns, pre, post,
                                  comp, delay, w, steps);
        if (!r || orc_set_input_raster(r, N, steps, raster) != 0 || orc_step(r, steps) != 0)
            return 1;
        if (orc_n_spikes(r) != nspk) return 1;
        total += (long)nspk;
        free(raster);
        free(spk);
        orc_destroy(r);
        orc_destroy(o);
    }
    printf("spikes %ld\n", total);
    free(off); free(parent); free(len); free(diam); free(mech); free(det); free(iext);
    free(pre); free(post); free(comp); free(delay); free(w);
    return 0;
}
