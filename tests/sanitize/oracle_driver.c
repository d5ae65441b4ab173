/*
 * Exercise every entry point of the oracle once, for a build with the
 * address and undefined-behaviour sanitizers (tests/test_sanitize.py). A
 * sanitizer report makes the run fail; the values are not checked here
 * (the pin tests do that).
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "../../oracle/cloak_oracle.h"

#define NR 96

static double lcg(uint64_t *s) {
    *s = *s * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(*s >> 11) * 0x1.0p-53;
}

int main(void) {
    uint64_t seed = 12345;
    double *in6 = malloc(sizeof(double) * 6 * NR), *out6 = malloc(sizeof(double) * 6 * NR);
    double *opl = malloc(sizeof(double) * NR), *hres = malloc(sizeof(double) * NR);
    double *trans = malloc(sizeof(double) * NR);
    int32_t *status = malloc(sizeof(int32_t) * NR);
    int64_t *nsteps = malloc(sizeof(int64_t) * NR);
    /* rays from a shell around the cloak towards points inside it: side, caps,
       metal end disks, misses */
    for (int i = 0; i < NR; i++) {
        double th = 2.0 * M_PI * lcg(&seed), el = (lcg(&seed) - 0.5) * 2.4;
        double o[3] = { 6.0 * cos(th) * cos(el), 6.0 * sin(th) * cos(el), 2.0 + 6.0 * sin(el) };
        double t[3] = { 2.4 * (lcg(&seed) - 0.5), 2.4 * (lcg(&seed) - 0.5), 4.4 * lcg(&seed) - 0.2 };
        for (int k = 0; k < 3; k++) {
            in6[k * NR + i] = o[k];
            in6[(3 + k) * NR + i] = t[k] - o[k];
        }
    }
    double total = 0.0;
    for (int axis = 0; axis < 2; axis++) {
        orc_cloak c = { 1.0, 2.0, 0.0, 4.0, axis, 1 };
        for (int scheme = 0; scheme < 3; scheme++) {
            orc_opts o = { scheme, 4, scheme == ORC_DP45 ? 1e-2 : 2e-3, 1e-8, 1e-8, 0.5, 3.0, 200000 };
            for (int br = 0; br < 2; br++) {
                orc_trace(&c, &o, br, NR, in6, out6, opl, status, hres, nsteps, trans);
                for (int i = 0; i < NR; i++) total += trans[i] + (double)status[i];
            }
        }
        orc_opts o = { ORC_DP45, 4, 1e-2, 1e-8, 1e-8, 0.5, 3.0, 200000 };
        orc_camera cam = { { 8.0, 1.0, 4.0 }, { 0.0, 0.0, 2.0 }, { 0.0, 0.0, 1.0 }, 40.0, 12, 10, 4, 7 };
        orc_room room = { { -10, -10, 0 }, { 10, 10, 10 }, 0.5, { { { 0 } } } };
        for (int f = 0; f < 6; f++)
            for (int p = 0; p < 2; p++)
                for (int k = 0; k < 3; k++) room.rgb[f][p][k] = 0.1f * (float)(f + p + k);
        enum { NS = 12 * 10 * 4 };
        int64_t ids[NS];
        for (int i = 0; i < NS; i++) ids[i] = i;
        uint8_t code[NS], code3[3 * NS];
        double rec[7 * NS], wimg[NS], wg[NS], w3[3 * NS], ray[3 * 6 * NR], wr[3 * NR];
        int32_t st[NS];
        for (int br = 0; br < 2; br++) {
            orc_render_samples(&c, &o, &room, &cam, 0, br, NS, ids, code, rec, st, wimg);
            orc_render_samples(NULL, &o, &room, &cam, 0, br, NS, ids, code, rec, st, wimg);
            for (int g = 0; g < 2; g++) orc_render_goggle(&c, &o, &cam, 0, br, g, NS, ids, wg);
            for (int g = -1; g < 2; g++)
                orc_render_reflections(&c, &o, &room, &cam, 0, br, g, NS, ids, w3, code3);
            orc_trace_reflections(&c, &o, br, NR, in6, wr, ray);
            for (int i = 0; i < NS; i++) total += wimg[i] + wg[i] + code[i] + w3[i];
        }
    }
    /* interface solves at random axes, normals and directions */
    for (int i = 0; i < 200; i++) {
        double ch[3], n[3] = { 0, 0, 1 }, k[3], e[3], T[2], R, Tt, Rr[2];
        for (int j = 0; j < 3; j++) { ch[j] = lcg(&seed) - 0.5; k[j] = lcg(&seed) - 0.5; e[j] = lcg(&seed) - 0.5; }
        double l = sqrt(ch[0] * ch[0] + ch[1] * ch[1] + ch[2] * ch[2]);
        for (int j = 0; j < 3; j++) ch[j] /= l;
        k[2] = -fabs(k[2]) - 0.05;
        l = sqrt(k[0] * k[0] + k[1] * k[1] + k[2] * k[2]);
        for (int j = 0; j < 3; j++) k[j] /= l;
        double eo = 0.5 + 4.0 * lcg(&seed), ee = 0.5 + 4.0 * lcg(&seed);
        if (orc_fresnel_in(eo, ee, ch, n, k, T, &R) == 0) total += T[0] + T[1] + R;
        if (orc_fresnel_in_pol(eo, ee, ch, n, k, e, T, &R) == 0) total += T[0] + T[1] + R;
        double kc[3] = { -k[0], -k[1], -k[2] };
        if (orc_fresnel_out(eo, ee, ch, n, kc, i & 1, &Tt, Rr) == 0) total += Tt + Rr[0] + Rr[1];
    }
    printf("oracle driver ok %.6e\n", total);
    free(in6); free(out6); free(opl); free(hres); free(trans); free(status); free(nsteps);
    return 0;
}
