/* Runs the oracle's entry points on one scene read from a file, for the
 * sanitizer test: every output buffer is allocated at exactly its size, so an
 * AddressSanitizer build reports any write outside it.
 *
 * Input file: int64 nv, nt, n; double R; float32 positions [nv][3]; uint32
 * triangles [nt][3]; float32 oriented points [n][3]; float32 normals [n][3].
 * Output file: uint32 row-range images [n][64][64], uint8 flags [n][64][64],
 * uint32 brute-force images, uint32 ranks [n] (each image ranked against all),
 * int64 distance matrix [n][n]. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_rici_rowrange(const float*, uint32_t, const uint32_t*, uint32_t, const float*, const float*, uint32_t,
                         float, uint32_t*, uint8_t*, uint64_t*, int);
int oracle_rici_rowrange_f64(const double*, uint32_t, const uint32_t*, uint32_t, const double*, const double*,
                             uint32_t, double, uint32_t*, uint8_t*, uint64_t*, int);
int oracle_rici_brute(const float*, uint32_t, const uint32_t*, uint32_t, const float*, const float*, uint32_t, float,
                      uint32_t*, uint8_t*, int);
int oracle_rank(const uint32_t*, uint32_t, const uint32_t*, uint32_t, const uint32_t*, uint32_t*, int64_t*, int);
int oracle_distance_matrix(const uint32_t*, uint32_t, const uint32_t*, uint32_t, int64_t*, int);

static void* take(FILE* f, size_t bytes)
{
    void* p = malloc(bytes ? bytes : 1);
    if (!p || fread(p, 1, bytes, f) != bytes) { fprintf(stderr, "short input\n"); exit(2); }
    return p;
}

int main(int argc, char** argv)
{
    if (argc != 3) return 2;
    FILE* f = fopen(argv[1], "rb");
    if (!f) return 2;
    int64_t hdr[3];
    double R;
    if (fread(hdr, sizeof hdr, 1, f) != 1 || fread(&R, sizeof R, 1, f) != 1) return 2;
    const uint32_t nv = (uint32_t)hdr[0], nt = (uint32_t)hdr[1], n = (uint32_t)hdr[2];
    float* pos = take(f, (size_t)nv * 3 * sizeof(float));
    uint32_t* tri = take(f, (size_t)nt * 3 * sizeof(uint32_t));
    float* op = take(f, (size_t)n * 3 * sizeof(float));
    float* nrm = take(f, (size_t)n * 3 * sizeof(float));
    fclose(f);

    const size_t px = (size_t)n * 64 * 64;
    uint32_t* img = malloc(px * sizeof(uint32_t));
    uint8_t* fl = malloc(px);
    uint64_t* wk = malloc((size_t)n * 5 * sizeof(uint64_t));
    uint32_t* img64 = malloc(px * sizeof(uint32_t));
    uint8_t* fl64 = malloc(px);
    uint32_t* brute = malloc(px * sizeof(uint32_t));
    uint8_t* flb = malloc(px);
    uint32_t* rank = malloc((size_t)n * sizeof(uint32_t));
    int64_t* dstar = malloc((size_t)n * sizeof(int64_t));
    uint32_t* tidx = malloc((size_t)n * sizeof(uint32_t));
    int64_t* mat = malloc((size_t)n * n * sizeof(int64_t));
    double* posd = malloc((size_t)nv * 3 * sizeof(double));
    double* opd = malloc((size_t)n * 3 * sizeof(double));
    double* nrmd = malloc((size_t)n * 3 * sizeof(double));
    for (size_t i = 0; i < (size_t)nv * 3; ++i) posd[i] = pos[i];
    for (size_t i = 0; i < (size_t)n * 3; ++i) { opd[i] = op[i]; nrmd[i] = nrm[i]; }
    for (uint32_t i = 0; i < n; ++i) tidx[i] = (i * 7u + 3u) % n;

    int rc = 0;
    rc |= oracle_rici_rowrange(pos, nv, tri, nt, op, nrm, n, (float)R, img, fl, wk, 4);
    rc |= oracle_rici_rowrange_f64(posd, nv, tri, nt, opd, nrmd, n, R, img64, fl64, NULL, 3);
    rc |= oracle_rici_brute(pos, nv, tri, nt, op, nrm, n, (float)R, brute, flb, 2);
    rc |= oracle_rank(img, n, img, n, tidx, rank, dstar, 4);
    rc |= oracle_distance_matrix(img, n, img, n, mat, 3);
    for (size_t i = 0; i < px; ++i)
        if (img[i] != img64[i] || fl[i] != fl64[i]) { fprintf(stderr, "f32 and f64 entries differ\n"); rc |= 4; break; }

    FILE* o = fopen(argv[2], "wb");
    if (!o) return 2;
    fwrite(img, sizeof(uint32_t), px, o);
    fwrite(fl, 1, px, o);
    fwrite(brute, sizeof(uint32_t), px, o);
    fwrite(rank, sizeof(uint32_t), n, o);
    fwrite(mat, sizeof(int64_t), (size_t)n * n, o);
    fclose(o);
    free(pos); free(tri); free(op); free(nrm); free(img); free(fl); free(wk); free(img64); free(fl64);
    free(brute); free(flb); free(rank); free(dstar); free(tidx); free(mat); free(posd); free(opd); free(nrmd);
    return rc;
}
