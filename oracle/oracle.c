/*
 * FP64 reference renderer for textured planar Gaussians — TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg may call this
 * code. It shares nothing with the HIP library: no headers, no helpers, no tables.
 *
 * It is a plain per-pixel definition of what the method computes, in double precision:
 *   - planar 2D Gaussian primitives P(u,v) = p + s_u t_u u + s_v t_v v      (Sec. 3.1, Eq. 1)
 *   - exact ray-plane intersection giving the local (u,v) of a pixel        (Sec. 3.1-3.2)
 *   - Gaussian value G = exp(-(u^2+v^2)/2), alpha = o G                     (Eq. 2, Sec. 3.1)
 *   - front-to-back blending in the global depth order                      (Eq. 3, Eq. 8)
 *   - texture coordinates s = (u+S)/(2S), t = (v+S)/(2S), S = 3             (Eq. 5)
 *   - bilinear texture filtering per primitive                              (Eq. 4, Eq. 6)
 *   - texture variants: tangent normals stored as two components with
 *     n_z = sqrt(max(0, 1 - n_x^2 - n_y^2)) rebuilt after filtering          (Sec. 3.5.1)
 *     per-primitive texture resolution and trilinear filtering over a box-filtered mip chain
 *     (the adaptive allocation and mipmapping the paper names as open)      (Sec. 5)
 *   - tangent normal rotated to world space, n = R n^t                      (Eq. 7)
 *   - G-buffers X = [albedo, metallic, roughness, normal]                   (Eq. 9)
 *   - split-sum shading L_o = L_d + L_s against an environment cubemap      (Eq. 10-12)
 *   - the indirect term: per-splat indirect radiance from spherical harmonics, blended as a
 *     fifth G-buffer map L_ind, and the visibility-weighted specular mix
 *     BRDF_LUT (V L_dir + (1 - V) L_ind)                                     (Eq. 9, Eq. 12)
 *   - the pre-integrated tables the shading reads: diffuse irradiance, roughness-prefiltered
 *     specular levels and the 2D BRDF lookup table                         (Sec. 3.5.4)
 * Every splat is tested against every pixel (no tiles, no culling grid).
 *
 * Readings of points the paper leaves open (also listed in the design notes):
 *   alpha = min(alpha_max, o G), splats with alpha < alpha_min are skipped, blending stops
 *   before the first splat whose transmittance would fall below t_min; the kernel support is
 *   the square max(|u|,|v|) <= S; texel centres sit at (i+1/2)/T with clamp-to-edge inside
 *   each primitive; the per-view order is the camera-space depth of the centre rounded to
 *   float32 (the precision the sort keys use), ties by splat index; splats with depth <=
 *   near_z are dropped; normals flip per splat to face the camera; shading uses the blended
 *   maps as they are (premultiplied), F0 = 0.04 (1-M) + albedo M, and an empty pixel takes
 *   the background colour; cube lookups use the OpenGL major-axis face rule with ties going
 *   X, then Y, then Z, bilinear at texel centres inside the face with clamp-to-edge.
 *   Indirect light: splat k carries real spherical-harmonic coefficients (orthonormal basis,
 *   no Condon-Shortley phase, degree <= 3) per colour channel, evaluated once per view at the
 *   mirror reflection of the camera-to-centre direction about the splat's plane and clamped
 *   at zero; the blended L_ind enters the shading premultiplied like the other maps, and V is
 *   a per-pixel input (V = 1 and no indirect map give the plain split sum).
 *
 * Decisions a tiny rounding difference can flip (support edge, alpha cut-off, termination,
 * grazing rays, cube-face ties) are recorded per pixel; for each flippable one the pixel is
 * re-rendered with that decision flipped, and both results are returned.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

#define OR_MAX_ALT 4

/* ------------------------------------------------------------------------------------- */
/* small vector helpers                                                                   */
/* ------------------------------------------------------------------------------------- */
static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static void normalize3(double* a) {
    double n = sqrt(dot3(a, a));
    if (n > 0) { a[0] /= n; a[1] /= n; a[2] /= n; }
}

/* rotation matrix (row-major) of the unit quaternion q = (w,x,y,z) */
static void quat_to_rot(const double* q, double* R) {
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

/* ------------------------------------------------------------------------------------- */
/* cube maps: OpenGL face selection and texel directions                                  */
/* faces 0..5 = +X,-X,+Y,-Y,+Z,-Z; texel [face][row t][col s][3]                           */
/* ------------------------------------------------------------------------------------- */
/* face and (s,t) in [0,1]^2 of direction d; *gap = relative gap between the two largest
   axis magnitudes (small means a face tie) */
static int cube_face_st(const double* d, double* s, double* t, double* gap) {
    double ax = fabs(d[0]), ay = fabs(d[1]), az = fabs(d[2]);
    int face; double sc, tc, ma;
    if (ax >= ay && ax >= az) {
        ma = ax;
        if (d[0] >= 0) { face = 0; sc = -d[2]; tc = -d[1]; } else { face = 1; sc = d[2]; tc = -d[1]; }
        *gap = (ax - (ay > az ? ay : az)) / (ax > 0 ? ax : 1);
    } else if (ay >= az) {
        ma = ay;
        if (d[1] >= 0) { face = 2; sc = d[0]; tc = d[2]; } else { face = 3; sc = d[0]; tc = -d[2]; }
        *gap = (ay - (ax > az ? ax : az)) / ay;
    } else {
        ma = az;
        if (d[2] >= 0) { face = 4; sc = d[0]; tc = -d[1]; } else { face = 5; sc = -d[0]; tc = -d[1]; }
        *gap = (az - (ax > ay ? ax : ay)) / az;
    }
    if (ma == 0) { *s = 0.5; *t = 0.5; *gap = 0; return 4; }
    *s = 0.5 * (sc / ma + 1.0);
    *t = 0.5 * (tc / ma + 1.0);
    return face;
}

/* unit direction through the centre of texel (i,j) of face f at resolution r */
static void cube_texel_dir(int f, int i, int j, int r, double* d) {
    double sc = 2.0 * (i + 0.5) / r - 1.0, tc = 2.0 * (j + 0.5) / r - 1.0;
    switch (f) {
        case 0: d[0] = 1;   d[1] = -tc; d[2] = -sc; break;
        case 1: d[0] = -1;  d[1] = -tc; d[2] = sc;  break;
        case 2: d[0] = sc;  d[1] = 1;   d[2] = tc;  break;
        case 3: d[0] = sc;  d[1] = -1;  d[2] = -tc; break;
        case 4: d[0] = sc;  d[1] = -tc; d[2] = 1;   break;
        default: d[0] = -sc; d[1] = -tc; d[2] = -1; break;
    }
    normalize3(d);
}

/* exact solid angle of texel (i,j) of a cube face at resolution r */
static double area_elem(double x, double y) { return atan2(x * y, sqrt(x * x + y * y + 1.0)); }
static double texel_solid_angle(int i, int j, int r) {
    double x0 = 2.0 * i / r - 1.0, x1 = 2.0 * (i + 1) / r - 1.0;
    double y0 = 2.0 * j / r - 1.0, y1 = 2.0 * (j + 1) / r - 1.0;
    return area_elem(x1, y1) - area_elem(x0, y1) - area_elem(x1, y0) + area_elem(x0, y0);
}

/* bilinear inside one face, texel centres at (i+1/2)/r, clamp-to-edge */
static void face_bilinear(const double* cube, int r, int face, double s, double t, double* out) {
    double X = s * r - 0.5, Y = t * r - 0.5;
    double fx0 = floor(X), fy0 = floor(Y);
    double fx = X - fx0, fy = Y - fy0;
    int i0 = (int)fx0, j0 = (int)fy0, i1 = i0 + 1, j1 = j0 + 1;
    if (i0 < 0) i0 = 0; if (i0 > r - 1) i0 = r - 1;
    if (i1 < 0) i1 = 0; if (i1 > r - 1) i1 = r - 1;
    if (j0 < 0) j0 = 0; if (j0 > r - 1) j0 = r - 1;
    if (j1 < 0) j1 = 0; if (j1 > r - 1) j1 = r - 1;
    const double* F = cube + (size_t)face * r * r * 3;
    for (int c = 0; c < 3; c++) {
        double a = F[((size_t)j0 * r + i0) * 3 + c], b = F[((size_t)j0 * r + i1) * 3 + c];
        double cc = F[((size_t)j1 * r + i0) * 3 + c], d = F[((size_t)j1 * r + i1) * 3 + c];
        out[c] = (1 - fy) * ((1 - fx) * a + fx * b) + fy * ((1 - fx) * cc + fx * d);
    }
}

static double cube_lookup(const double* cube, int r, const double* dir, double* out) {
    double s, t, gap;
    int f = cube_face_st(dir, &s, &t, &gap);
    face_bilinear(cube, r, f, s, t, out);
    return gap;
}

/* ------------------------------------------------------------------------------------- */
/* pre-integrated tables (Sec. 3.5.4: pre-integrated diffuse irradiance, roughness-selected */
/* specular levels, precomputed 2D BRDF lookup)                                           */
/* ------------------------------------------------------------------------------------- */

/* Irradiance E(n) = sum over source texels of L(w) max(0, n.w) dOmega, at the texel centres
   of an out_res cube. */
int or_irradiance(const float* env, int r, int out_res, double* out) {
    int nsrc = 6 * r * r;
    double* dirs = (double*)malloc(sizeof(double) * 3 * nsrc);
    double* dw = (double*)malloc(sizeof(double) * nsrc);
    if (!dirs || !dw) { free(dirs); free(dw); return -1; }
    for (int f = 0; f < 6; f++)
        for (int j = 0; j < r; j++)
            for (int i = 0; i < r; i++) {
                int k = (f * r + j) * r + i;
                cube_texel_dir(f, i, j, r, dirs + 3 * k);
                dw[k] = texel_solid_angle(i, j, r);
            }
    int nout = 6 * out_res * out_res;
#pragma omp parallel for schedule(dynamic, 4)
    for (int o = 0; o < nout; o++) {
        int f = o / (out_res * out_res), rem = o % (out_res * out_res);
        int j = rem / out_res, i = rem % out_res;
        double n[3];
        cube_texel_dir(f, i, j, out_res, n);
        double acc[3] = {0, 0, 0};
        for (int k = 0; k < nsrc; k++) {
            double c = dot3(n, dirs + 3 * k);
            if (c <= 0) continue;
            double w = c * dw[k];
            acc[0] += w * env[3 * k + 0];
            acc[1] += w * env[3 * k + 1];
            acc[2] += w * env[3 * k + 2];
        }
        out[3 * o + 0] = acc[0]; out[3 * o + 1] = acc[1]; out[3 * o + 2] = acc[2];
    }
    free(dirs); free(dw);
    return 0;
}

/* GGX normal distribution with alpha = roughness^2 */
static double ggx_D(double ndh, double a) {
    double a2 = a * a;
    double d = ndh * ndh * (a2 - 1.0) + 1.0;
    return a2 / (M_PI * d * d);
}

/* Specular level l (l >= 1) at roughness l/(L-1), resolution r >> l: with N = V = R (the
   reflection direction r), the expectation that the importance-sampled GGX prefilter estimates,
       pref(r) = sum_j L_j (r.w_j)^+ D(h_j) dOmega_j / sum_j (r.w_j)^+ D(h_j) dOmega_j,
       h_j = normalize(r + w_j),
   evaluated exactly over the source (level 0) texels. Level 0 is the environment itself.
   out holds the levels one after another, each [6][r_l][r_l][3]. */
int or_prefilter(const float* env, int r, int levels, double* out) {
    int nsrc = 6 * r * r;
    for (int k = 0; k < nsrc * 3; k++) out[k] = env[k];
    if (levels <= 1) return 0;
    double* dirs = (double*)malloc(sizeof(double) * 3 * nsrc);
    double* dw = (double*)malloc(sizeof(double) * nsrc);
    if (!dirs || !dw) { free(dirs); free(dw); return -1; }
    for (int f = 0; f < 6; f++)
        for (int j = 0; j < r; j++)
            for (int i = 0; i < r; i++) {
                int k = (f * r + j) * r + i;
                cube_texel_dir(f, i, j, r, dirs + 3 * k);
                dw[k] = texel_solid_angle(i, j, r);
            }
    size_t off = (size_t)nsrc * 3;
    for (int l = 1; l < levels; l++) {
        int rl = r >> l;
        if (rl < 1) rl = 1;
        double rough = (double)l / (levels - 1);
        double a = rough * rough;
        int nout = 6 * rl * rl;
        double* dst = out + off;
#pragma omp parallel for schedule(dynamic, 4)
        for (int o = 0; o < nout; o++) {
            int f = o / (rl * rl), rem = o % (rl * rl);
            int j = rem / rl, i = rem % rl;
            double n[3];
            cube_texel_dir(f, i, j, rl, n);
            double acc[3] = {0, 0, 0}, wsum = 0;
            for (int k = 0; k < nsrc; k++) {
                const double* w = dirs + 3 * k;
                double c = dot3(n, w);
                if (c <= 0) continue;
                double h[3] = {n[0] + w[0], n[1] + w[1], n[2] + w[2]};
                normalize3(h);
                double wt = c * ggx_D(dot3(n, h), a) * dw[k];
                acc[0] += wt * env[3 * k + 0];
                acc[1] += wt * env[3 * k + 1];
                acc[2] += wt * env[3 * k + 2];
                wsum += wt;
            }
            dst[3 * o + 0] = acc[0] / wsum;
            dst[3 * o + 1] = acc[1] / wsum;
            dst[3 * o + 2] = acc[2] / wsum;
        }
        off += (size_t)nout * 3;
    }
    free(dirs); free(dw);
    return 0;
}

static double radical_inverse2(uint32_t b) {
    b = (b << 16) | (b >> 16);
    b = ((b & 0x55555555u) << 1) | ((b & 0xAAAAAAAAu) >> 1);
    b = ((b & 0x33333333u) << 2) | ((b & 0xCCCCCCCCu) >> 2);
    b = ((b & 0x0F0F0F0Fu) << 4) | ((b & 0xF0F0F0F0u) >> 4);
    b = ((b & 0x00FF00FFu) << 8) | ((b & 0xFF00FF00u) >> 8);
    return (double)b * 2.3283064365386963e-10; /* 2^-32 */
}

/* Split-sum BRDF table (Karis 2013): for N.V = (i+1/2)/n and roughness (j+1/2)/n,
     A = mean over samples of (1 - Fc) G_vis,  B = mean of Fc G_vis,
   with half vectors importance-sampled from GGX (alpha = roughness^2) at the Hammersley
   points (k/S, radical_inverse(k)), Fc = (1 - V.H)^5, G_vis = G V.H / (N.H N.V), G the
   Smith-Schlick term with k = alpha/2. out[j][i][2]. */
int or_brdf_lut(int n, int samples, double* out) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int j = 0; j < n; j++) {
        double rough = (j + 0.5) / n;
        double a = rough * rough;
        double kk = a / 2.0;
        for (int i = 0; i < n; i++) {
            double nv = (i + 0.5) / n;
            double V[3] = {sqrt(1.0 - nv * nv), 0.0, nv};
            double A = 0, B = 0;
            for (int s = 0; s < samples; s++) {
                double xi1 = (double)s / samples, xi2 = radical_inverse2((uint32_t)s);
                double phi = 2.0 * M_PI * xi1;
                double ct = sqrt((1.0 - xi2) / (1.0 + (a * a - 1.0) * xi2));
                double st = sqrt(fmax(0.0, 1.0 - ct * ct));
                double H[3] = {st * cos(phi), st * sin(phi), ct};
                double vh = dot3(V, H);
                double L[3] = {2 * vh * H[0] - V[0], 2 * vh * H[1] - V[1], 2 * vh * H[2] - V[2]};
                double nl = L[2] > 0 ? L[2] : 0, nh = H[2] > 0 ? H[2] : 0;
                if (vh < 0) vh = 0;
                if (nl > 0) {
                    double g1v = nv / (nv * (1 - kk) + kk), g1l = nl / (nl * (1 - kk) + kk);
                    double gvis = g1v * g1l * vh / (nh * nv);
                    double fc = pow(1.0 - vh, 5.0);
                    A += (1 - fc) * gvis;
                    B += fc * gvis;
                }
            }
            out[(j * n + i) * 2 + 0] = A / samples;
            out[(j * n + i) * 2 + 1] = B / samples;
        }
    }
    return 0;
}

static void lut_lookup(const double* lut, int n, double x, double y, double* ab) {
    double X = x * n - 0.5, Y = y * n - 0.5;
    double fx0 = floor(X), fy0 = floor(Y), fx = X - fx0, fy = Y - fy0;
    int i0 = (int)fx0, j0 = (int)fy0, i1 = i0 + 1, j1 = j0 + 1;
    if (i0 < 0) i0 = 0; if (i0 > n - 1) i0 = n - 1;
    if (i1 < 0) i1 = 0; if (i1 > n - 1) i1 = n - 1;
    if (j0 < 0) j0 = 0; if (j0 > n - 1) j0 = n - 1;
    if (j1 < 0) j1 = 0; if (j1 > n - 1) j1 = n - 1;
    for (int c = 0; c < 2; c++) {
        double a = lut[(j0 * n + i0) * 2 + c], b = lut[(j0 * n + i1) * 2 + c];
        double cc = lut[(j1 * n + i0) * 2 + c], d = lut[(j1 * n + i1) * 2 + c];
        ab[c] = (1 - fy) * ((1 - fx) * a + fx * b) + fy * ((1 - fx) * cc + fx * d);
    }
}

/* ------------------------------------------------------------------------------------- */
/* scene / camera / parameter blocks                                                      */
/* ------------------------------------------------------------------------------------- */
typedef struct {
    double R[9], t[3];            /* world -> camera, row-major */
    double fx, fy, cx, cy;
    double o[3];                  /* camera centre in world space */
    double Rc2w[9];
} cam_t;

/* params: [0] S, [1] alpha_min, [2] alpha_max, [3] t_min, [4] near_z, [5..7] bg,
           [8] ambiguity margin (relative), [9] grazing threshold on |cos| */
typedef struct {
    double S, amin, amax, tmin, near_z, bg[3], eps, graze;
} par_t;

typedef struct {
    const double* spec; int spec_res, levels;  /* levels one after another */
    const double* irr; int irr_res;
    const double* lut; int lut_res;
} env_t;

typedef struct {
    int n, T;
    const float *means, *quats, *scales, *opac, *tex;
    const int32_t* chart_of;
    int fmt;                 /* 0: 8 channels per texel (normal xyz); 1: 7 channels (normal xy) */
    int tri;                 /* 1: trilinear filtering over the chart's mip chain */
    const int32_t* ctab;     /* [n_charts][2] level-0 texel offset and log2 T of each chart;
                                NULL: every chart is T x T, chart c at texel c T^2 */
} scene_t;

typedef struct {
    int keep;                 /* 0 when culled by the near plane */
    float depth32;            /* camera depth rounded to float32: the sort key */
    double mu[3], tu[3], tv[3], n[3], R[9];
    double su, sv, op, sigma;
} splat_t;

static void make_cam(const double* c, cam_t* cam) {
    for (int k = 0; k < 3; k++) {
        for (int m = 0; m < 3; m++) cam->R[k * 3 + m] = c[k * 4 + m];
        cam->t[k] = c[k * 4 + 3];
    }
    cam->fx = c[12]; cam->fy = c[13]; cam->cx = c[14]; cam->cy = c[15];
    for (int k = 0; k < 3; k++)
        for (int m = 0; m < 3; m++) cam->Rc2w[k * 3 + m] = cam->R[m * 3 + k];
    for (int k = 0; k < 3; k++)
        cam->o[k] = -(cam->Rc2w[k * 3 + 0] * cam->t[0] + cam->Rc2w[k * 3 + 1] * cam->t[1] +
                      cam->Rc2w[k * 3 + 2] * cam->t[2]);
}

static void make_par(const double* p, par_t* par) {
    par->S = p[0]; par->amin = p[1]; par->amax = p[2]; par->tmin = p[3]; par->near_z = p[4];
    par->bg[0] = p[5]; par->bg[1] = p[6]; par->bg[2] = p[7]; par->eps = p[8]; par->graze = p[9];
}

/* Step 1 of the definition, per splat: rotation, frame, depth, facing sign. */
static void setup_splat(const scene_t* sc, const cam_t* cam, const par_t* par, int k, splat_t* s) {
    double q[4];
    for (int m = 0; m < 4; m++) q[m] = sc->quats[4 * k + m];
    double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int m = 0; m < 4; m++) q[m] /= qn;
    quat_to_rot(q, s->R);
    for (int m = 0; m < 3; m++) {
        s->mu[m] = sc->means[3 * k + m];
        s->tu[m] = s->R[m * 3 + 0];
        s->tv[m] = s->R[m * 3 + 1];
        s->n[m] = s->R[m * 3 + 2];
    }
    s->su = sc->scales[2 * k + 0];
    s->sv = sc->scales[2 * k + 1];
    s->op = sc->opac[k];
    double z = cam->R[6] * s->mu[0] + cam->R[7] * s->mu[1] + cam->R[8] * s->mu[2] + cam->t[2];
    s->depth32 = (float)z;
    s->keep = z > par->near_z;
    double om[3] = {cam->o[0] - s->mu[0], cam->o[1] - s->mu[1], cam->o[2] - s->mu[2]};
    s->sigma = dot3(s->n, om) >= 0 ? 1.0 : -1.0;
}

/* Texel (i,j) of mip level l of a chart whose level 0 is T x T texels at P (C channels per
   texel): level l is the mean of the 2^l x 2^l block of level-0 texels it covers (the box
   filter the chain is defined by; level 0 is the texture itself). */
static void mip_texel(const float* P, int T, int C, int l, int i, int j, double* v) {
    int b = 1 << l;
    for (int c = 0; c < C; c++) v[c] = 0.0;
    for (int jj = j * b; jj < (j + 1) * b; jj++)
        for (int ii = i * b; ii < (i + 1) * b; ii++)
            for (int c = 0; c < C; c++) v[c] += P[((size_t)jj * T + ii) * C + c];
    for (int c = 0; c < C; c++) v[c] /= (double)b * b;
}

/* Bilinear at (s,t) on mip level l (T_l = T >> l texels a side): texel centres at
   (i+1/2)/T_l, clamp-to-edge inside the chart (Eq. 6). */
static void bilinear_level(const float* P, int T, int C, int l, double s, double t, double* a) {
    int Tl = T >> l;
    double X = s * Tl - 0.5, Y = t * Tl - 0.5;
    double fx0 = floor(X), fy0 = floor(Y), fx = X - fx0, fy = Y - fy0;
    int i0 = (int)fx0, j0 = (int)fy0, i1 = i0 + 1, j1 = j0 + 1;
    if (i0 < 0) i0 = 0; if (i0 > Tl - 1) i0 = Tl - 1;
    if (i1 < 0) i1 = 0; if (i1 > Tl - 1) i1 = Tl - 1;
    if (j0 < 0) j0 = 0; if (j0 > Tl - 1) j0 = Tl - 1;
    if (j1 < 0) j1 = 0; if (j1 > Tl - 1) j1 = Tl - 1;
    double v00[8], v10[8], v01[8], v11[8];
    mip_texel(P, T, C, l, i0, j0, v00);
    mip_texel(P, T, C, l, i1, j0, v10);
    mip_texel(P, T, C, l, i0, j1, v01);
    mip_texel(P, T, C, l, i1, j1, v11);
    for (int c = 0; c < C; c++)
        a[c] = (1 - fy) * ((1 - fx) * v00[c] + fx * v10[c]) + fy * ((1 - fx) * v01[c] + fx * v11[c]);
}

/* Texture value of primitive k at (s,t), as 8 channels (albedo 3, roughness, normal xyz,
   metallic). rho = texture footprint of one pixel in level-0 texels of a unit-resolution
   chart (scaled by the chart's T below); used only with trilinear filtering, whose level is
   lambda = log2(T rho): below 0 the level-0 bilinear sample, else the blend of levels
   floor(lambda) and floor(lambda)+1 by the fraction, the last level alone beyond it. With
   two-component normals the third is rebuilt after filtering. */
static void tex_sample(const scene_t* sc, int k, double s, double t, double rho, double* a) {
    int chart = sc->chart_of[k];
    int C = sc->fmt ? 7 : 8;
    int T = sc->T;
    size_t off = (size_t)chart * T * T;
    if (sc->ctab) { off = (size_t)sc->ctab[2 * chart]; T = 1 << sc->ctab[2 * chart + 1]; }
    const float* P = sc->tex + off * C;
    double v[8];
    int L = 0;
    while ((1 << L) < T) L++;              /* levels 0..L, T = 2^L */
    double lam = sc->tri ? log2(T * rho) : 0.0;
    if (!sc->tri || !(lam > 0.0)) {
        bilinear_level(P, T, C, 0, s, t, v);
    } else {
        int l0 = (int)floor(lam);
        if (l0 >= L) {
            bilinear_level(P, T, C, L, s, t, v);
        } else {
            double f = lam - l0, v1[8];
            bilinear_level(P, T, C, l0, s, t, v);
            bilinear_level(P, T, C, l0 + 1, s, t, v1);
            for (int c = 0; c < C; c++) v[c] = (1 - f) * v[c] + f * v1[c];
        }
    }
    if (sc->fmt) {
        /* stored (albedo 3, roughness, n_x, n_y, metallic) */
        for (int c = 0; c < 6; c++) a[c] = v[c];
        a[6] = sqrt(fmax(0.0, 1.0 - v[4] * v[4] - v[5] * v[5]));
        a[7] = v[6];
    } else {
        for (int c = 0; c < 8; c++) a[c] = v[c];
    }
}

/* ------------------------------------------------------------------------------------- */
/* shading (Eq. 10-12: split sum, specular mix of direct and indirect light by V)         */
/* ------------------------------------------------------------------------------------- */
#define OR_GB 11   /* G-buffer channels: albedo 3, metallic, roughness, normal 3, L_ind 3 */

/* g = [albedo r,g,b, metallic, roughness, normal x,y,z, L_ind r,g,b] (blended), A = alpha,
   V = visibility, dir = world ray direction through the pixel centre. Returns the smallest
   cube-face gap. */
static double shade(const env_t* env, const par_t* par, const double* g, double A, double V,
                    const double* dir, double* C) {
    if (A <= 0.0) { C[0] = par->bg[0]; C[1] = par->bg[1]; C[2] = par->bg[2]; return 1.0; }
    double wo[3] = {-dir[0], -dir[1], -dir[2]};
    normalize3(wo);
    double N[3] = {g[5], g[6], g[7]};
    double nn = sqrt(dot3(N, N));
    if (nn > 0) { N[0] /= nn; N[1] /= nn; N[2] /= nn; }
    else { N[0] = wo[0]; N[1] = wo[1]; N[2] = wo[2]; }
    double ndv = dot3(N, wo);
    double wr[3] = {2 * ndv * N[0] - wo[0], 2 * ndv * N[1] - wo[1], 2 * ndv * N[2] - wo[2]};
    double M = g[3], Rg = g[4];
    double E[3];
    double gap = cube_lookup(env->irr, env->irr_res, N, E);
    double rc = Rg < 0 ? 0 : (Rg > 1 ? 1 : Rg);
    double lev = rc * (env->levels - 1);
    int l0 = (int)floor(lev);
    if (l0 > env->levels - 1) l0 = env->levels - 1;
    int l1 = l0 + 1 < env->levels ? l0 + 1 : env->levels - 1;
    double fl = lev - l0;
    double P0[3], P1[3];
    const double* lvl = env->spec;
    const double *s0 = NULL, *s1 = NULL;
    int r0 = 0, r1 = 0;
    for (int l = 0; l < env->levels; l++) {
        int rl = env->spec_res >> l;
        if (rl < 1) rl = 1;
        if (l == l0) { s0 = lvl; r0 = rl; }
        if (l == l1) { s1 = lvl; r1 = rl; }
        lvl += (size_t)6 * rl * rl * 3;
    }
    double g2 = cube_lookup(s0, r0, wr, P0);
    if (g2 < gap) gap = g2;
    cube_lookup(s1, r1, wr, P1);
    double ab[2];
    double ndvc = ndv < 0 ? 0 : (ndv > 1 ? 1 : ndv);
    lut_lookup(env->lut, env->lut_res, ndvc, rc, ab);
    for (int c = 0; c < 3; c++) {
        double Lp = (1 - fl) * P0[c] + fl * P1[c];
        double F0 = 0.04 * (1 - M) + g[c] * M;
        double Ld = g[c] / M_PI * (1 - M) * E[c];
        double Lmix = V * Lp + (1 - V) * g[8 + c];
        C[c] = Ld + Lmix * (F0 * ab[0] + ab[1]) + (1 - A) * par->bg[c];
    }
    return gap;
}

/* ------------------------------------------------------------------------------------- */
/* one pixel                                                                              */
/* ------------------------------------------------------------------------------------- */
typedef struct { float key; int k; double alpha, u, v, rho; } cand_t;

static int cand_cmp(const void* a, const void* b) {
    const cand_t* x = (const cand_t*)a;
    const cand_t* y = (const cand_t*)b;
    if (x->key < y->key) return -1;
    if (x->key > y->key) return 1;
    return (x->k > y->k) - (x->k < y->k);
}

typedef struct { int k, kind; } flip_t;   /* kind 0: inclusion of splat k, 1: stop at splat k */

typedef struct {
    double rgba[4], gbuf[OR_GB];
    int n_blend, n_support, graze;
    double min_gap;
    double sens;       /* sum over G-buffer channels of max_rgb |dC/dg_c| (shading condition) */
    int n_amb;
    flip_t amb[OR_MAX_ALT];
} pix_out_t;

static void pixel_ray(const cam_t* cam, int x, int y, double* d) {
    double dc[3] = {(x + 0.5 - cam->cx) / cam->fx, (y + 0.5 - cam->cy) / cam->fy, 1.0};
    for (int m = 0; m < 3; m++)
        d[m] = cam->Rc2w[m * 3 + 0] * dc[0] + cam->Rc2w[m * 3 + 1] * dc[1] + cam->Rc2w[m * 3 + 2] * dc[2];
}

static void note_amb(pix_out_t* po, int k, int kind) {
    if (po->n_amb < OR_MAX_ALT) { po->amb[po->n_amb].k = k; po->amb[po->n_amb].kind = kind; }
    po->n_amb++;
}

/* Render pixel (x,y). flip (may be NULL) forces the opposite outcome of one decision;
   record != 0 records the near-threshold decisions in po. cand is scratch of n entries.
   lind (may be NULL) = per-splat indirect radiance [n][3] of this view; V = visibility. */
static void render_pixel(const scene_t* sc, const splat_t* sp, const cam_t* cam, const par_t* par,
                         const env_t* env, const double* lind, double V, int x, int y,
                         const flip_t* flip, int record, cand_t* cand, pix_out_t* po) {
    double d[3];
    pixel_ray(cam, x, y, d);
    double dn = sqrt(dot3(d, d));
    int nc = 0;
    po->n_support = 0; po->graze = 0; po->n_amb = 0; po->min_gap = 1.0;
    for (int k = 0; k < sc->n; k++) {
        const splat_t* s = sp + k;
        if (!s->keep) continue;
        double den = dot3(d, s->n);
        if (den == 0.0) continue;
        double mo[3] = {s->mu[0] - cam->o[0], s->mu[1] - cam->o[1], s->mu[2] - cam->o[2]};
        double lam = dot3(mo, s->n) / den;
        if (lam <= 0.0) continue;
        double P[3] = {cam->o[0] + lam * d[0] - s->mu[0], cam->o[1] + lam * d[1] - s->mu[1],
                       cam->o[2] + lam * d[2] - s->mu[2]};
        double u = dot3(P, s->tu) / s->su, v = dot3(P, s->tv) / s->sv;
        double m = fmax(fabs(u), fabs(v));
        int in_support = m <= par->S;
        int amb_s = fabs(m - par->S) <= par->eps * par->S;
        if (!in_support && !amb_s) continue;       /* outside the support, not near its edge */
        double oG = s->op * exp(-0.5 * (u * u + v * v));
        double alpha = oG < par->amax ? oG : par->amax;
        int pass_alpha = alpha >= par->amin;
        int include = in_support && pass_alpha;
        if (record) {
            int amb_a = oG < par->amax && fabs(oG - par->amin) <= par->eps * par->amin;
            /* one flipped comparison changes the inclusion only if the other test passes */
            if ((amb_s && pass_alpha) || (amb_a && in_support)) note_amb(po, k, 0);
            if (include && fabs(den) / dn < par->graze) po->graze = 1;
        }
        if (flip && flip->kind == 0 && flip->k == k) include = !include;
        if (in_support) po->n_support++;
        if (!include) continue;
        cand[nc].key = s->depth32; cand[nc].k = k; cand[nc].alpha = alpha; cand[nc].u = u; cand[nc].v = v;
        cand[nc].rho = 0.0;
        if (sc->tri) {
            /* footprint of the pixel on the texture: derivatives of (s,t) = ((u,v)+S)/(2S)
               along the image axes, from the ray d(X,Y) = R^T ((X-cx)/fx, (Y-cy)/fy, 1),
               lambda = ((mu-o).n)/(d.n) and P = o + lambda d - mu */
            double J[2][2];
            for (int ax = 0; ax < 2; ax++) {
                double dd[3];
                for (int m = 0; m < 3; m++)
                    dd[m] = cam->Rc2w[m * 3 + ax] / (ax == 0 ? cam->fx : cam->fy);
                double dlam = -lam * dot3(dd, s->n) / den;
                double dP[3] = {lam * dd[0] + dlam * d[0], lam * dd[1] + dlam * d[1],
                                lam * dd[2] + dlam * d[2]};
                J[ax][0] = dot3(dP, s->tu) / s->su / (2 * par->S);
                J[ax][1] = dot3(dP, s->tv) / s->sv / (2 * par->S);
            }
            double rx = sqrt(J[0][0] * J[0][0] + J[0][1] * J[0][1]);
            double ry = sqrt(J[1][0] * J[1][0] + J[1][1] * J[1][1]);
            cand[nc].rho = rx > ry ? rx : ry;
        }
        nc++;
    }
    qsort(cand, nc, sizeof(cand_t), cand_cmp);
    double T = 1.0;
    double g[OR_GB];
    for (int m = 0; m < OR_GB; m++) g[m] = 0.0;
    int nb = 0;
    for (int c = 0; c < nc; c++) {
        const splat_t* s = sp + cand[c].k;
        double a = cand[c].alpha;
        double Tn = T * (1.0 - a);
        int stop = Tn < par->tmin;
        if (record && fabs(Tn - par->tmin) <= par->eps * par->tmin) note_amb(po, cand[c].k, 1);
        if (flip && flip->kind == 1 && flip->k == cand[c].k) stop = !stop;
        if (stop) break;
        double w = a * T;
        double tx[8];
        double ss = (cand[c].u + par->S) / (2 * par->S), tt = (cand[c].v + par->S) / (2 * par->S);
        tex_sample(sc, cand[c].k, ss, tt, cand[c].rho, tx);
        double nt[3] = {tx[4], tx[5], tx[6]};
        double l = sqrt(dot3(nt, nt));
        if (l > 0) { nt[0] /= l; nt[1] /= l; nt[2] /= l; } else { nt[0] = 0; nt[1] = 0; nt[2] = 1; }
        double nw[3];
        for (int m = 0; m < 3; m++)
            nw[m] = s->sigma * (s->R[m * 3 + 0] * nt[0] + s->R[m * 3 + 1] * nt[1] + s->R[m * 3 + 2] * nt[2]);
        g[0] += w * tx[0]; g[1] += w * tx[1]; g[2] += w * tx[2];
        g[3] += w * tx[7];
        g[4] += w * tx[3];
        g[5] += w * nw[0]; g[6] += w * nw[1]; g[7] += w * nw[2];
        if (lind) {
            const double* li = lind + 3 * (size_t)cand[c].k;
            g[8] += w * li[0]; g[9] += w * li[1]; g[10] += w * li[2];
        }
        T = Tn;
        nb++;
    }
    double A = 1.0 - T;
    for (int m = 0; m < OR_GB; m++) po->gbuf[m] = g[m];
    po->rgba[3] = A;
    po->n_blend = nb;
    double gap = 1.0;
    po->sens = 0.0;
    if (env) {
        gap = shade(env, par, g, A, V, d, po->rgba);
        if (record && A > 0.0) {
            /* central differences of the shading in each G-buffer channel: how much a rounding
               of the blended maps moves the shaded radiance */
            for (int c = 0; c < OR_GB; c++) {
                double h = 1e-7, gp[OR_GB], gm[OR_GB], Cp[4], Cm[4];
                for (int m = 0; m < OR_GB; m++) { gp[m] = g[m]; gm[m] = g[m]; }
                gp[c] += h; gm[c] -= h;
                shade(env, par, gp, A, V, d, Cp);
                shade(env, par, gm, A, V, d, Cm);
                double mx = 0;
                for (int m = 0; m < 3; m++) mx = fmax(mx, fabs(Cp[m] - Cm[m]) / (2 * h));
                po->sens += mx;
            }
        }
    } else { po->rgba[0] = po->rgba[1] = po->rgba[2] = 0; }
    po->min_gap = gap;
}

/* ------------------------------------------------------------------------------------- */
/* exported entry points                                                                  */
/* ------------------------------------------------------------------------------------- */

/* Per-splat step for one camera: depth rounded to float32 (the sort key), the keep flag,
   the facing sign. */
int or_splat_setup(int n, const float* means, const float* quats, const float* scales,
                   const float* opac, const double* cam16, const double* params,
                   float* depth32, int32_t* keep, double* sigma) {
    scene_t sc = {n, 1, means, quats, scales, opac, NULL, NULL, 0, 0, NULL};
    cam_t cam; par_t par;
    make_cam(cam16, &cam); make_par(params, &par);
    for (int k = 0; k < n; k++) {
        splat_t s;
        setup_splat(&sc, &cam, &par, k, &s);
        depth32[k] = s.depth32; keep[k] = s.keep; sigma[k] = s.sigma;
    }
    return 0;
}

/*
 * Render the listed pixels (pix = [P][2] x,y).
 * tex: level-0 texels, [n_charts][T][T][C] or, with ctab, charts of 2^ctab[2c+1] texels a
 * side at texel offsets ctab[2c]; C = 8 (fmt 0) or 7 (fmt 1: albedo 3, roughness, n_x, n_y,
 * metallic); tri = 1 filters trilinearly over the box-filtered mip chain.
 * lind [n][3] per-splat indirect radiance of this view (or NULL: no indirect map),
 * vis [P] visibility per listed pixel (or NULL: V = 1).
 * out_rgba [P][4], out_gbuf [P][11] (albedo 3, metallic, roughness, normal 3, L_ind 3),
 * out_stat [P][7]: n_blend, n_support, n_amb, grazing flag, min cube-face gap, n_alt,
 *                  shading sensitivity (sum over channels of max_rgb |dC/dg_c|),
 * alt_rgba [P][OR_MAX_ALT][4], alt_gbuf [P][OR_MAX_ALT][11] (the first n_alt are valid).
 * env_spec == NULL renders G-buffers only (rgb = 0).
 */
int or_render(int n, int T, const float* means, const float* quats, const float* scales,
              const float* opac, const float* tex, const int32_t* chart_of,
              int fmt, int tri, const int32_t* ctab,
              const double* cam16, const double* params,
              const double* env_spec, int spec_res, int spec_levels,
              const double* env_irr, int irr_res, const double* env_lut, int lut_res,
              const double* lind, const double* vis, const int32_t* pix, int P,
              double* out_rgba, double* out_gbuf, double* out_stat,
              double* alt_rgba, double* alt_gbuf) {
    scene_t sc = {n, T, means, quats, scales, opac, tex, chart_of, fmt, tri, ctab};
    cam_t cam; par_t par;
    make_cam(cam16, &cam); make_par(params, &par);
    env_t envs = {env_spec, spec_res, spec_levels, env_irr, irr_res, env_lut, lut_res};
    const env_t* env = env_spec ? &envs : NULL;
    splat_t* sp = (splat_t*)malloc(sizeof(splat_t) * (n > 0 ? n : 1));
    if (!sp) return -1;
    for (int k = 0; k < n; k++) setup_splat(&sc, &cam, &par, k, sp + k);
    int err = 0;
#pragma omp parallel
    {
        cand_t* cand = (cand_t*)malloc(sizeof(cand_t) * (n > 0 ? n : 1));
        if (!cand) {
#pragma omp atomic write
            err = -1;
        }
#pragma omp for schedule(dynamic, 16)
        for (int p = 0; p < P; p++) {
            if (!cand) continue;
            int x = pix[2 * p], y = pix[2 * p + 1];
            double V = vis ? vis[p] : 1.0;
            pix_out_t po;
            render_pixel(&sc, sp, &cam, &par, env, lind, V, x, y, NULL, 1, cand, &po);
            for (int m = 0; m < 4; m++) out_rgba[4 * p + m] = po.rgba[m];
            for (int m = 0; m < OR_GB; m++) out_gbuf[OR_GB * p + m] = po.gbuf[m];
            int nalt = po.n_amb < OR_MAX_ALT ? po.n_amb : OR_MAX_ALT;
            double* st = out_stat + 7 * p;
            st[0] = po.n_blend; st[1] = po.n_support; st[2] = po.n_amb; st[3] = po.graze;
            st[4] = po.min_gap; st[5] = nalt; st[6] = po.sens;
            for (int a = 0; a < nalt; a++) {
                pix_out_t pa;
                render_pixel(&sc, sp, &cam, &par, env, lind, V, x, y, &po.amb[a], 0, cand, &pa);
                for (int m = 0; m < 4; m++) alt_rgba[(p * OR_MAX_ALT + a) * 4 + m] = pa.rgba[m];
                for (int m = 0; m < OR_GB; m++)
                    alt_gbuf[(p * OR_MAX_ALT + a) * OR_GB + m] = pa.gbuf[m];
            }
        }
        free(cand);
    }
    free(sp);
    return err;
}

/* Shade a given G-buffer: gbuf [P][11], alpha [P], vis [P] (or NULL: V = 1),
   pixels [P][2] -> rgb [P][3]. */
int or_shade(const double* gbuf, const double* alpha, const double* vis, const int32_t* pix, int P,
             const double* cam16, const double* params,
             const double* env_spec, int spec_res, int spec_levels,
             const double* env_irr, int irr_res, const double* env_lut, int lut_res,
             double* out_rgb, double* out_gap) {
    cam_t cam; par_t par;
    make_cam(cam16, &cam); make_par(params, &par);
    env_t env = {env_spec, spec_res, spec_levels, env_irr, irr_res, env_lut, lut_res};
#pragma omp parallel for schedule(static)
    for (int p = 0; p < P; p++) {
        double d[3], C[4];
        pixel_ray(&cam, pix[2 * p], pix[2 * p + 1], d);
        double gap = shade(&env, &par, gbuf + OR_GB * p, alpha[p], vis ? vis[p] : 1.0, d, C);
        out_rgb[3 * p + 0] = C[0]; out_rgb[3 * p + 1] = C[1]; out_rgb[3 * p + 2] = C[2];
        if (out_gap) out_gap[p] = gap;
    }
    return 0;
}

/* Bilinear cube lookups (for tests): dirs [P][3] -> out [P][3]. */
int or_cube_sample(const double* cube, int r, const double* dirs, int P, double* out) {
    for (int p = 0; p < P; p++) cube_lookup(cube, r, dirs + 3 * p, out + 3 * p);
    return 0;
}

/* Texel directions and solid angles of one cube resolution (for tests). */
int or_cube_texels(int r, double* dirs, double* solid) {
    for (int f = 0; f < 6; f++)
        for (int j = 0; j < r; j++)
            for (int i = 0; i < r; i++) {
                int k = (f * r + j) * r + i;
                cube_texel_dir(f, i, j, r, dirs + 3 * k);
                solid[k] = texel_solid_angle(i, j, r);
            }
    return 0;
}

/* LUT bilinear lookups (for tests): xy [P][2] -> ab [P][2]. */
int or_lut_sample(const double* lut, int n, const double* xy, int P, double* ab) {
    for (int p = 0; p < P; p++) lut_lookup(lut, n, xy[2 * p], xy[2 * p + 1], ab + 2 * p);
    return 0;
}

/* ------------------------------------------------------------------------------------- */
/* indirect light from per-splat spherical harmonics (Sec. 3.5-3.6, Eq. 9 and 12)         */
/* ------------------------------------------------------------------------------------- */
/* Associated Legendre function P_l^m(x), m >= 0, without the Condon-Shortley phase:
   P_m^m = (2m-1)!! (1-x^2)^(m/2), P_{m+1}^m = (2m+1) x P_m^m, then the three-term recurrence
   (l-m) P_l^m = (2l-1) x P_{l-1}^m - (l+m-1) P_{l-2}^m. */
static double legendre_p(int l, int m, double x) {
    double pmm = 1.0, st = sqrt(fmax(0.0, 1.0 - x * x));
    for (int i = 1; i <= m; i++) pmm *= (2.0 * i - 1.0) * st;
    if (l == m) return pmm;
    double p1 = (2.0 * m + 1.0) * x * pmm;
    if (l == m + 1) return p1;
    double p0 = pmm, pl = p1;
    for (int ll = m + 2; ll <= l; ll++) {
        pl = ((2.0 * ll - 1.0) * x * p1 - (ll + m - 1.0) * p0) / (ll - m);
        p0 = p1; p1 = pl;
    }
    return pl;
}

static double factorial(int k) { double f = 1.0; for (int i = 2; i <= k; i++) f *= i; return f; }

/* Real orthonormal spherical harmonic Y_{l,m} at unit direction d (index l*l + l + m):
   K = sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!), Y = K P_l^0(cos th) for m = 0,
   sqrt(2) K P_l^m(cos th) cos(m phi) for m > 0, sqrt(2) K P_l^|m|(cos th) sin(|m| phi) for m < 0,
   with cos th = d_z and phi = atan2(d_y, d_x). */
static double sh_real(int l, int m, const double* d) {
    double r = sqrt(dot3(d, d));
    double ct = d[2] / r, ph = atan2(d[1], d[0]);
    int am = m < 0 ? -m : m;
    double K = sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * factorial(l - am) / factorial(l + am));
    double P = legendre_p(l, am, ct);
    if (m == 0) return K * P;
    if (m > 0) return sqrt(2.0) * K * P * cos(am * ph);
    return sqrt(2.0) * K * P * sin(am * ph);
}

/* Basis values for tests: dirs [P][3] -> out [P][(degree+1)^2]. */
int or_sh_basis(int degree, const double* dirs, int P, double* out) {
    if (degree < 0 || degree > 3) return -1;
    int K = (degree + 1) * (degree + 1);
    for (int p = 0; p < P; p++)
        for (int l = 0; l <= degree; l++)
            for (int m = -l; m <= l; m++) out[(size_t)p * K + l * l + l + m] = sh_real(l, m, dirs + 3 * p);
    return 0;
}

/* Per-splat indirect radiance for one camera: sh [n][(degree+1)^2][3] coefficients; the
   direction is the mirror reflection w_r = d - 2 (d.n) n of the unit camera-to-centre
   direction d about the splat normal n (the third column of R; the sign of n does not
   matter); out [n][3] = max(0, sum_j c_j Y_j(w_r)) per channel. */
int or_indirect_eval(int n, const float* means, const float* quats, const float* sh, int degree,
                     const double* cam16, double* out) {
    if (degree < 0 || degree > 3) return -1;
    int K = (degree + 1) * (degree + 1);
    cam_t cam;
    make_cam(cam16, &cam);
    for (int k = 0; k < n; k++) {
        double q[4], R[9];
        for (int m = 0; m < 4; m++) q[m] = quats[4 * k + m];
        double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
        for (int m = 0; m < 4; m++) q[m] /= qn;
        quat_to_rot(q, R);
        double nrm[3] = {R[2], R[5], R[8]};
        double d[3] = {means[3 * k + 0] - cam.o[0], means[3 * k + 1] - cam.o[1],
                       means[3 * k + 2] - cam.o[2]};
        normalize3(d);
        double dn = dot3(d, nrm);
        double wr[3] = {d[0] - 2 * dn * nrm[0], d[1] - 2 * dn * nrm[1], d[2] - 2 * dn * nrm[2]};
        double acc[3] = {0, 0, 0};
        for (int l = 0; l <= degree; l++)
            for (int m = -l; m <= l; m++) {
                int j = l * l + l + m;
                double Y = sh_real(l, m, wr);
                for (int c = 0; c < 3; c++) acc[c] += sh[((size_t)k * K + j) * 3 + c] * Y;
            }
        for (int c = 0; c < 3; c++) out[3 * (size_t)k + c] = acc[c] > 0 ? acc[c] : 0.0;
    }
    return 0;
}

/* Thread count of the OpenMP loops above (n > 0 sets it); returns the count in effect. Used
   only to time the oracle on a given number of host cores. */
int or_set_threads(int n) {
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
}
