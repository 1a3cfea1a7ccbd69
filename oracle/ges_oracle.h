/*
 * ges_oracle.h -- plain, slow CPU oracle for the GES tile rasterizer.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this file; only tests, the smoke check and the CPU-baseline leg of the
 * benchmark use it.  It shares no code with the HIP library.
 *
 * What it computes (GES, arXiv 2402.10128):
 *   - per-splat preprocess: view transform, 3-D covariance from scale and
 *     rotation with the scales multiplied by the approximate modification
 *     phi_rho(beta) (Sec. 4.2, Eq. approx; Sec. 4.1 for Sigma from S and R),
 *     EWA projection Sigma' = J W Sigma W^T J^T (Sec. 4.1), conic, screen
 *     radius, alpha-floor threshold, tile rectangle, SH colour (Sec. 4.1);
 *   - (tile, depth) keys, a stable sort and per-tile ranges;
 *   - per-pixel front-to-back alpha compositing over the depth-sorted splats of
 *     the pixel's tile, the discrete form of the volume-rendering integral
 *     (Sec. 4.2, Eq. transimttance), with either the paper's approximate
 *     rasterization (falloff exp(-q/2) on the phi-scaled covariance, "PHI") or
 *     the exact GES exponent exp(-q^(beta/2)/2) of Eq. ges ("GEF");
 *   - the reverse-mode gradient of that compositing w.r.t. every 2-D splat
 *     quantity (mean2D, conic, opacity, colour, beta).
 *
 * Two arithmetic modes:
 *   OC_MODE_F32: the canonical binary32 operation sequence (no FMA contraction,
 *     correctly rounded division and sqrt, canonical exp/log defined below) for
 *     every value that feeds an integer decision; compositing in binary64 from
 *     those binary32 values.
 *   OC_MODE_F64: everything in binary64 with libm exp/log.
 *
 * Every function returns 0 on success, a negative value on bad arguments.
 */
#ifndef GES_ORACLE_H
#define GES_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

enum { OC_MODE_F32 = 0, OC_MODE_F64 = 1 };
enum { OC_FALLOFF_PHI = 0, OC_FALLOFF_GEF = 1, OC_FALLOFF_PHI_EXACT = 2 };
enum { OC_TILES_SQUARE = 0, OC_TILES_ELLIPSE = 1 };
enum { OC_TILE = 16 };

typedef struct {
  int64_t n;
  int32_t sh_degree;              /* 0..3 */
  const float* means;             /* [n,3] */
  const float* log_scales;        /* [n,3] */
  const float* quats;             /* [n,4] (w,x,y,z), not necessarily unit */
  const float* opacity_logits;    /* [n] */
  const float* sh;                /* [n,(D+1)^2,3] */
  const float* beta;              /* [n] true beta (2 = Gaussian) */
} oc_splats;

typedef struct {
  int32_t width, height;
  float R[9];                     /* world->camera rotation, row-major; x right, y down, z forward */
  float t[3];
  float fx, fy, cx, cy;           /* pixel (i,j) has its centre at (i,j) */
  float near_z;
} oc_camera;

typedef struct {
  int32_t falloff;                /* OC_FALLOFF_* */
  int32_t tile_cull;              /* OC_TILES_* */
  float rho;                      /* shape strength of phi_rho (0.1 in the paper) */
  float bg[3];
} oc_params;

/* Per-splat projected record, binary64 storage.  In F32 mode every float
 * field holds an exact binary32 value. */
typedef struct {
  double* u;            /* [n] mean2D x (pixels) */
  double* v;            /* [n] mean2D y */
  double* depth;        /* [n] camera-space z */
  double* conic;        /* [n,3] inverse 2-D covariance (a,b,c): q = a dx^2 + 2 b dx dy + c dy^2 */
  double* qmax;         /* [n] alpha-floor threshold in quadratic-form units */
  double* opacity;      /* [n] sigmoid(logit) */
  double* rgb;          /* [n,3] clamped SH colour */
  double* beta;         /* [n] the splat's beta (copied; used by the GEF falloff) */
  int32_t* radius;      /* [n] screen radius in pixels, 0 if culled */
  int32_t* rect;        /* [n,4] tx0,ty0,tx1,ty1 inclusive tile bounds */
  int64_t* tiles_touched;/* [n] number of tiles the splat is listed in (0 = culled) */
  uint8_t* clamp_bits;  /* [n] bit0..2: rgb channel clamped at 0; bit3/4: x/y guard clamp in J */
} oc_record;

/* Canonical binary32 exp / log (used by the F32 mode), exposed for tests. */
void oc_exp_c(const float* x, float* y, int64_t n);
void oc_log_c(const float* x, float* y, int64_t n);
void oc_lgamma_c(const float* x, float* y, int64_t n);

int oc_preprocess(int mode, const oc_splats* s, const oc_camera* cam, const oc_params* p, oc_record* out);

/* Is tile (tx,ty) in splat i's tile set?  (rect membership, plus the ellipse test in ELLIPSE mode) */
int oc_splat_in_tile(int mode, const oc_record* r, int64_t i, const oc_camera* cam, const oc_params* p,
                     int32_t tx, int32_t ty);

/* Per-tile entry counts (number of splats listed in each tile), tiles row-major. */
int oc_tile_counts(int mode, const oc_record* r, int64_t n, const oc_camera* cam, const oc_params* p,
                   int64_t* counts);

/* All (tile, splat) entries: duplication order (splats in index order, tiles row-major in the rect),
 * key = (tile << 32) | bits(float(depth)), then a stable sort by key and tile ranges [start,end)
 * (empty tile -> (0,0)).  keys/values hold num_keys entries (sum of tiles_touched). */
int oc_build_keys(int mode, const oc_record* r, int64_t n, const oc_camera* cam, const oc_params* p,
                  uint64_t* keys, uint32_t* values, int64_t num_keys, int64_t* ranges);

/* Sorted list of one tile (ascending depth, ties by splat index); *len receives the length;
 * at most cap entries are written. */
int oc_tile_list(int mode, const oc_record* r, int64_t n, const oc_camera* cam, const oc_params* p,
                 int32_t tile, uint32_t* out, int64_t cap, int64_t* len);

typedef struct {
  int64_t pairs_examined;   /* splats visited per pixel up to (and including) the terminating one */
  int64_t pairs_skipped;    /* ... of which failed the alpha-floor test */
  int64_t pairs_blended;    /* ... of which were composited */
  int64_t pixels_flagged;   /* pixels whose termination decision lies within the flag margin */
  uint64_t decision_hash;   /* hash of every composite / clamp / termination decision */
} oc_stats;

/* Forward render of the pixels of the listed tiles.  lists: values[] with per-tile [start,end) in
 * ranges (indexed by tile id).  tiles == NULL renders every tile.  Outputs are full images [H,W,(3)];
 * pixels of tiles not rendered are left untouched.  alt receives, for flagged pixels, the colour of
 * the other branch of the termination decision (else a copy of the primary colour). */
int oc_render(int mode, const oc_record* r, int64_t n, const oc_camera* cam, const oc_params* p,
              const uint32_t* values, const int64_t* ranges, const int32_t* tiles, int64_t n_tiles,
              double* img, double* final_T, int32_t* n_contrib, uint8_t* flags, double* alt,
              oc_stats* stats);

/* The same compositing without tiles: every pixel walks all visible splats in (depth, index) order. */
int oc_render_untiled(int mode, const oc_record* r, int64_t n, const oc_camera* cam, const oc_params* p,
                      double* img, double* final_T, int32_t* n_contrib, uint8_t* flags, double* alt,
                      oc_stats* stats);

/* Reverse-mode gradient of the rendered image w.r.t. the per-splat 2-D quantities, for the pixels of
 * the listed tiles.  dL_dimg [H,W,3].  g2d [n,10] accumulates (not overwritten):
 * (u, v, a, b, c, opacity, r, g, b, beta); the beta column is non-zero only in GEF mode.
 * delta [n,10] (nullable) accumulates, over pixels whose termination test (within 1e-3 relative of
 * 1e-4) or alpha clamp (o G within 1e-5 of 0.99) is ambiguous in floating point, the absolute
 * difference between the gradients of the two branches of that decision.
 * mass [n,10] (nullable) accumulates the sum of |per-pixel contribution|, the scale of the rounding
 * error of summing the contributions in binary32.
 * ebound [n,10] (nullable) accumulates a first-order bound on the error of each per-pixel
 * contribution when it is evaluated in binary32 with one-ulp exp2/log2/reciprocal and the
 * transmittance recovered back to front by division (running error analysis; model in the source). */
int oc_backward(int mode, const oc_record* r, int64_t n, const oc_camera* cam, const oc_params* p,
                const uint32_t* values, const int64_t* ranges, const int32_t* tiles, int64_t n_tiles,
                const double* dL_dimg, double* g2d, double* delta, double* mass, double* ebound,
                oc_stats* stats);

/* Untiled reverse pass: every pixel walks all visible splats in (depth, index) order. */
int oc_backward_untiled(int mode, const oc_record* r, int64_t n, const oc_camera* cam, const oc_params* p,
                        const double* dL_dimg, double* g2d, double* delta, double* mass, double* ebound,
                        oc_stats* stats);

int oc_num_threads(void);
/* Threads of the following OpenMP loops (n > 0). */
void oc_set_num_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
