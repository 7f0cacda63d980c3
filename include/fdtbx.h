/*
 * fdtbx -- fibre-diffraction profile quadrature on AMD Instinct MI355X (gfx950).
 *
 * C ABI of the hot path of "FDTBX - Computational Tools for Simulation of X-ray
 * Fiber Diffraction Patterns from Atomic Coordinates": reflection enumeration,
 * direct structure factors, per-reflection shell quadrature of the broadened
 * profile at the query points of flat-detector pixels, Lorentz correction, and
 * the adjoint of that image.
 *
 * Conventions (all entry points):
 *   - Lengths in Angstrom, reciprocal lengths in 1/Angstrom, angles in radians
 *     (the tutorial passes cell angles in radians); detector distance and pixel
 *     pitch share one length unit (millimetres in the examples).
 *   - Laboratory frame of the tutorial's "Unit cell and reciprocal-space frame":
 *     crystal c along +z (the fibre axis), b in the yz-plane; the beam runs along
 *     a* = +x, normal to the fibre (the notebook's check |beam . fibre| <= 1e-3
 *     holds exactly).  The fibre may be tilted toward the beam (fdtbx_geometry.tilt);
 *     the detector stays normal to the beam.
 *   - Detector images are float32 [height][width], row-major, row 0 at the bottom
 *     (origin='lower'); pixel (i, j) has its centre at
 *     y = (i + 1/2 - center_x) pixel, z = (j + 1/2 - center_y) pixel.
 *   - Pointers documented as "device" must be device memory of the current HIP
 *     device (hipMalloc or a torch CUDA tensor); "host" pointers are ordinary
 *     memory.  The caller owns every buffer; the library never allocates or frees.
 *   - Every call is asynchronous on `stream` (a hipStream_t; NULL is the null
 *     stream) unless it says it synchronises.  Argument checks run on the host
 *     before any launch; on error nothing is launched and no output is written.
 *   - Empty inputs are valid: with n_hkl = 0 images come out zero, culling lists
 *     empty and gradients zero, and the per-reflection pointers may be NULL; with
 *     n_atoms = 0 the structure factors are zero and the atom pointers may be NULL.
 *   - Return value 0 on success, a negative FDTBX_ERR_* code otherwise;
 *     fdtbx_error_string() describes it.  No exceptions cross the ABI.
 */
#ifndef FDTBX_H
#define FDTBX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  FDTBX_OK = 0,
  FDTBX_ERR_INVALID_ARGUMENT = -1, /* null pointer, negative size, widths both zero, NaN, ... */
  FDTBX_ERR_GEOMETRY = -2,         /* distance/pixel/wavelength <= 0, cell not a valid parallelepiped */
  FDTBX_ERR_BUFFER_TOO_SMALL = -3, /* an output or workspace capacity is too small; see the call */
  FDTBX_ERR_HIP = -4,              /* a HIP runtime call failed; fdtbx_last_hip_error() has the code */
  FDTBX_ERR_UNSUPPORTED = -5       /* a parameter outside what this build implements */
};

/* Unit cell (tutorial Table "unitcell"). */
typedef struct fdtbx_cell {
  double a, b, c;             /* edge lengths, A */
  double alpha, beta, gamma;  /* angles b^c, a^c, a^b, radians */
} fdtbx_cell;

/* Flat detector normal to the beam along lab x (tutorial Table "experiment").  The
 * fibre axis is lab z tilted by `tilt` about lab y (the detector horizontal) toward +x,
 * n = (sin tilt, 0, cos tilt); tilt 0 is the fibre normal to the beam.  A tilted fibre
 * makes the D term of Eq. harmonic nonzero; the pixel ring coordinates become
 * Z = S.n, R = |S - Z n| (see fdtbx_pixel_map). */
typedef struct fdtbx_geometry {
  double wavelength;          /* A */
  double distance;            /* sample-detector distance, same unit as pixel */
  double pixel;               /* pixel pitch */
  int32_t width, height;      /* pixels along lab y (horizontal) and lab z (vertical) */
  double center_x, center_y;  /* beam centre in pixel units (width/2, height/2 puts it between pixels) */
  double tilt;                /* fibre tilt, radians, |tilt| < pi/2 */
  int32_t tile_w;             /* pixel tile width: 2, 4, 8, 16 or 32 (0 means FDTBX_TILE); a tile
                                 is tile_w x (64 / tile_w) pixels, one pixel per lane of a wave */
  int32_t mirror;             /* bit 0: fold the left-right mirror symmetry, bit 1: the up-down
                                 (Friedel) symmetry (below); 0: every tile runs */
  int32_t tile_waves;         /* waves per tile of fdtbx_profile, fdtbx_profile_adjoint and
                                 fdtbx_profile_cyl: 1, 2 or 4 (wave w takes the chunks w, w + waves,
                                 ... of 64 pairs of the tile's list, or for the cylindrical average
                                 of 8 ring indices of each pair; the forward's first wave adds the
                                 others' pixel sums in wave order); 0: the library's choice, 4 when the
                                 launched tiles fit in eight rounds of one-wave workgroups (32 per
                                 compute unit), else 2.  The batched persistent kernels run one
                                 wave per (model, tile) item whatever the value */
  int32_t unit_pairs;         /* pairs per work unit of fdtbx_profile_balanced (and so of
                                 fdtbx_profile_pattern): 0 is the library's choice from the pair
                                 count (fdtbx_unit_pairs); the image depends on it in the last bits
                                 (the grouping of the sums), so two launches that must agree bit for
                                 bit (a folded and an unfolded one) fix it to the same value */
  double det_tilt;            /* detector tilt, radians, |det_tilt| < pi/2: the detector plane
                                 turned about its horizontal axis (through the beam centre) so that
                                 its top leans toward the sample for det_tilt > 0; pixel (y, z) then
                                 sits at X = (distance - z sin det_tilt, y, z cos det_tilt), which
                                 must lie in front of the sample (X_x > 0) for every row; 0 is a
                                 detector normal to the beam */
} fdtbx_geometry;
/* Mirror fold.  With center_x = width / 2 exactly, pixel (i, j) and its mirror (width-1-i, j)
 * have y of opposite sign and equal z, so their (R, Z) are bit-identical (R depends on y only
 * through y^2, for any tilt).  With width a multiple of tile_w, the mirror of a tile is a tile
 * with the same (R, Z) box, hence the same culling list, and the per-tile kernels compute the
 * same value for a pixel and its mirror.  mirror = 1 (which requires both conditions) makes
 * fdtbx_profile, fdtbx_profile_cyl and the batched forward run the left ceil(tiles_x / 2) tile
 * columns only and write each value to the pixel and its mirror (the image is bit-identical to
 * the unfolded one with the same waves per tile, fdtbx_launch_waves), and makes the adjoints
 * take grad(i, j) + grad(width-1-i, j) as the weight of the computed pixel.  fdtbx_pixel_map
 * still produces every tile; fdtbx_cull lists the launched columns only (the right columns'
 * lists are empty).
 *
 * Up-down (Friedel) fold, bit 1 of mirror.  With the fibre normal to the beam (tilt 0) and
 * center_y = height / 2 exactly, pixel (i, j) and (i, height-1-j) have z of opposite sign, so
 * their (R, Z) are (R, Z) and (R, -Z) bit for bit.  The reflection list is closed under
 * negation.  The mate -D of a reflection D has the same weight (|F|^2 by Friedel's law with
 * real form factors; the disorder and damping factors are even in hkl); its ring point at
 * (R, -Z) and its nodes are those of D at (R, Z) negated, with the same orientational weights
 * (the tangent frame of -D spans the same plane and the node grid is symmetric); and every
 * lineshape is even.  So the pattern obeys I(R, -Z) = I(R, Z) exactly in the model.  The per-tile
 * kernels then run the top ceil(tiles_y / 2) tile rows only (height must be a multiple of the
 * tile height 64 / tile_w, so tile row tiles_y-1-ty holds the mirror rows of row ty) and write
 * each value also to (i, height-1-j); with both bits, to all four mirror images.  Unlike the
 * left-right fold this is not bit-identical to the unfolded image: a mirrored pixel sums the
 * mates' contributions in another order, so the two agree to float32 rounding (the top rows
 * computed are bit-identical).  The adjoints take the sum of grad over the mirror images as
 * the weight of the computed pixel, and fdtbx_cull lists the launched rows only. */

/* Orientational and lattice disorder (section "Angular peak shapes", tutorial
 * Table "paracrystal").  sigma_theta: Gaussian standard deviation; gamma_theta:
 * Lorentzian HWHM; both zero is an error.  N_base: coherent cells along a, b, c
 * (non-integer allowed).  g: Hosemann relative spacing fluctuation per axis
 * (Eq. Ah).  intensity_model: 1 applies the intensity loss of Eq. Ipara, 0 omits it.
 * lineshape: per-axis peak of integral breadth 1/N_eff (Eq. Neff), unit integral per
 * lattice period and height N_eff, in u = a_i.(p - s):
 *   FDTBX_LINESHAPE_LAUE      N sinc^2(N u) (Eq. I_shape with N -> N_eff), support |u| <= m/N
 *   FDTBX_LINESHAPE_GAUSSIAN  N exp(-pi N^2 u^2) (matched integral breadth), support |u| <= m/N
 *   FDTBX_LINESHAPE_HOSEMANN  (1 - A^2)/(1 - 2 A cos(2 pi u) + A^2), A = max(0, (N-1)/(N+1))
 *                             (Eq. Z with breadth (1-A)/(1+A) = 1/N, Eq. breadth), support
 *                             |u| <= 1/2 (one lattice period; m unused)
 * B_axis: axis-dependent Debye-Waller damping (section "Paracrystalline disorder"), a factor
 * exp(-1/4 sum_i B_i (S.a_i/|a_i|)^2) on each reflection's intensity at S = D_hkl, A^2. */
#define FDTBX_LINESHAPE_LAUE 0
#define FDTBX_LINESHAPE_GAUSSIAN 1
#define FDTBX_LINESHAPE_HOSEMANN 2
typedef struct fdtbx_disorder {
  double sigma_theta, gamma_theta;
  double N_base[3];
  double g[3];
  int32_t intensity_model;
  int32_t lineshape;
  double B_axis[3];
} fdtbx_disorder;

/* Refinable globals of a model, in this order, for the gradient and update calls:
 * sigma_theta, gamma_theta, N_base a, b, c, g a, b, c, B_axis a, b, c. */
#define FDTBX_N_GLOBALS 11

/* Shell quadrature (section "Numerical evaluation: per-reflection shell quadrature"). */
typedef struct fdtbx_quadrature {
  int32_t n_nodes;    /* nodes per side of the midpoint (d1, d2) grid, 1..256 */
  double T;           /* grid half extent in tangent-plane units, 0 < T < 10 */
  double sigma_r;     /* radial shell width collapsed to its integral sigma_r sqrt(2 pi) */
  int32_t m;          /* Laue-kernel zeros kept per lattice axis, 1..8 */
  double delta;       /* Lorentz regulariser of Eq. lorentz, 1/A */
  double d_min, d_max;/* resolution shell, A; d_max <= 0: no low-resolution limit */
  double extinction;  /* skip hkl with 2 pi^2 sum_i g_i^2 h_i^2 above this (<= 0: never) */
} fdtbx_quadrature;

typedef struct fdtbx_model {
  fdtbx_cell cell;
  fdtbx_geometry geom;
  fdtbx_disorder dis;
  fdtbx_quadrature quad;
} fdtbx_model;

/* Description of the last error on this thread (static string, never NULL). */
const char* fdtbx_error_string(int code);
/* hipError_t of the last FDTBX_ERR_HIP on this thread. */
int fdtbx_last_hip_error(void);

/* ------------------------------------------------------------------ reflections
 * fdtbx_hkl_capacity: host only.  Upper bound on the number of reflections of
 * fdtbx_enumerate_hkl for this cell and d_min (size of the index box
 * |h| <= floor(a/d_min)+1, likewise k and l, since h = D.a).
 *
 * fdtbx_enumerate_hkl: every (h,k,l) != 0 with
 *   |D|^2 <= (1/d_min^2)(1 + 1e-9)  and  |D|^2 >= (1/d_max^2)(1 - 1e-9) (if d_max > 0),
 * D = h a* + k b* + l c* (Eq. laue3d, Eq. recip_basis), the resolution shell of the
 * tutorial's reflection list, in ascending lexicographic order of (h,k,l).  The
 * list is closed under negation, the mate of entry i being entry n-1-i.  The
 * predicate is evaluated in IEEE binary64 with a fixed operation order and no
 * fused multiply-add, so the list is reproducible bit for bit.
 *   extinction host float64 [4] = (g_a, g_b, g_c, limit) or NULL: also drop reflections
 *         with 2 pi^2 ((g_a^2 h^2 + g_b^2 k^2) + g_c^2 l^2) > limit, whose paracrystalline
 *         intensity loss prod_i A_i (Eq. Ah) is below exp(-limit); the kept list is
 *         still closed under negation and ordered
 *   hkl   device int32 [cap][3] output
 *   n_out device int64 [1] output: number of reflections written
 *   ws    device workspace of at least fdtbx_enumerate_workspace(cell, d_min) bytes */
int fdtbx_hkl_capacity(const fdtbx_cell* cell, double d_min, int64_t* cap);
size_t fdtbx_enumerate_workspace(const fdtbx_cell* cell, double d_min);
int fdtbx_enumerate_hkl(const fdtbx_cell* cell, double d_min, double d_max, const double* extinction,
                        int32_t* hkl, int64_t cap, int64_t* n_out, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------ structure factors
 * F_hkl = sum_j occ_j f_t(j)(s) exp(-B_j s^2) exp(2 pi i (h x_j + k y_j + l z_j))
 * (Eq. structure_factor with the isotropic Debye-Waller factor, B = 8 pi^2 <u^2>),
 * s = |D_hkl|/2 = sin(theta)/lambda, f_t(s) = sum_{g=1..4} a_g exp(-b_g s^2) + c.
 *   x, y, z  device float32 [n_atoms], fractional coordinates
 *   B, occ   device float32 [n_atoms]
 *   type     device int32 [n_atoms], 0 <= type < n_types (not checked on device)
 *   ff       device float32 [n_types][9] = a1..a4, b1..b4, c; n_types <= 16
 *   hkl      device int32 [n_hkl][3]
 *   F        device float32 [n_hkl][2] (re, im) output, may be NULL
 *   F2       device float32 [n_hkl] output |F|^2, may be NULL
 *   ws       device workspace of fdtbx_sf_workspace(n_hkl, n_atoms) bytes
 * Deterministic: fixed summation order, no atomics. */
size_t fdtbx_sf_workspace(int64_t n_hkl, int64_t n_atoms);
int fdtbx_structure_factors(const fdtbx_cell* cell, int64_t n_atoms, const float* x, const float* y,
                            const float* z, const float* B, const float* occ, const int32_t* type,
                            const float* ff, int32_t n_types, const int32_t* hkl, int64_t n_hkl, float* F,
                            float* F2, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------ pattern building blocks
 * Record layouts (device memory, produced and consumed by the library; exposed
 * so each step can be checked on its own).
 *
 * Reflection record, FDTBX_REFL_FLOATS float32 per reflection (see
 * fdtbx_reflection_prep).  Culling record, FDTBX_CULL_DOUBLES float64 per
 * reflection:
 *   [0..3]  R_lo, R_hi, Z_lo, Z_hi    box in (R, Z) of the query points it can reach
 *   [4..5]  P2_lo, P2_hi              range of |p|^2 (annulus about r0)
 *   [6..11] n1R, n1Z, rho1, n2R, n2Z, rho2   inward edge normals of the arc wedge and
 *                                     the support extent along each; rho1 < 0 disables
 * The support extents use the per-axis half-widths w_i of the lineshape's support in u:
 * 1/2 for the Hosemann lineshape, else m/N_eff,i bounded above (no transcendental) by
 * m (1/N_base,i + min(pi^2 g_i^2 h_i^2, 1)).
 *   [12]    1 if the reflection is kept (not removed by the extinction cull), else 0
 *   [13..15] reserved (0)
 * Node record, FDTBX_NODE_FLOATS float32 per node, node k = i2*n + i1:
 *   [0] c - 1   [1] c d1   [2] c d2   [3] omega   [4] d omega/d sigma_theta
 *   [5] d omega/d gamma_theta   [6] d1   [7] d2
 * with c = (1 + d1^2 + d2^2)^(-1/2), d_j = -T + (i_j + 1/2) h, h = 2T/n and
 * omega = sigma_r sqrt(2 pi) g(Delta) c^3 h^2, Delta = arccos c (Eq. node_weight
 * without the per-reflection r0^2).
 * The n^2 node records are followed by nb^2 block records, nb = ceil(n/FDTBX_NODE_BLOCK),
 * block b = b2*nb + b1 covering the nodes with i_j in [b_j B, b_j B + B) (B = FDTBX_NODE_BLOCK)
 * that exist:
 *   [0..2] centre c_j of the block's float32 values of (c - 1, c d1, c d2)
 *   [3]    max_j |c_j| + r_j
 *   [4..6] half-widths r_j, rounded up so every node value v_j satisfies |v_j - c_j| <= r_j
 *   [7]    0
 * The profile kernels test blocks before nodes; the records are derived data, not part
 * of the quadrature. */
#define FDTBX_REFL_FLOATS 64 /* 256 bytes: a per-pair cache line, then the rest */
#define FDTBX_CULL_DOUBLES 16
#define FDTBX_NODE_FLOATS 8
#define FDTBX_NODE_BLOCK 4
#define FDTBX_TILE 8 /* default pixel tile width (fdtbx_geometry.tile_w = 0): 8 x 8 tiles */

/* Host: the pixel-tile grid of a geometry, tiles_x = ceil(width / tile_w) columns and
 * tiles_y = ceil(height / (64 / tile_w)) rows; tile t covers columns (t % tiles_x) tile_w
 * onward and rows (t / tiles_x) (64 / tile_w) onward. */
int fdtbx_tile_grid(const fdtbx_geometry* geom, int32_t* tiles_x, int32_t* tiles_y);

/* Host: the waves per tile that fdtbx_profile and fdtbx_profile_adjoint use for this
 * geometry (its tile_waves, or the library's choice for its launched tiles on the current
 * device). */
int fdtbx_launch_waves(const fdtbx_geometry* geom, int32_t* waves);

/* Rows of FDTBX_NODE_FLOATS float32 in the node table of n_nodes per side:
 * n_nodes^2 + ceil(n_nodes/FDTBX_NODE_BLOCK)^2; 0 if n_nodes is outside 1..256. */
int64_t fdtbx_node_rows(int32_t n_nodes);

/* Node table of the shell quadrature (Eqs. gnomonic, node_weight; angular shape
 * of section "Angular peak shapes": Gaussian if gamma_theta = 0, Lorentzian if
 * sigma_theta = 0, otherwise the unit-peak Voigt profile, evaluated on the device
 * through the Faddeeva function w(z) by Weideman's rational series).
 *   nodes device float32 [fdtbx_node_rows(n_nodes)][FDTBX_NODE_FLOATS] output */
int fdtbx_node_table(const fdtbx_disorder* dis, const fdtbx_quadrature* quad, float* nodes, void* stream);

/* Per-reflection preparation (Eqs. Ah, Neff, Ipara, gnomonic; axis damping D):
 *   hkl  device int32 [n_hkl][3];  F2 device float32 [n_hkl] (|F|^2)
 *   refl device float32 [n_hkl][FDTBX_REFL_FLOATS] output (layout private to the
 *        profile kernels except: [0] W = |F|^2 I_para D, [1..3] N_eff a,b,c, [4] r0)
 *   cull device float64 [n_hkl][FDTBX_CULL_DOUBLES] output (layout above) */
int fdtbx_reflection_prep(const fdtbx_model* model, const int32_t* hkl, int64_t n_hkl, const float* F2,
                          float* refl, double* cull, void* stream);

/* Ring coordinates of every pixel and the (R, Z) boxes of the pixel tiles.
 *   pix  device float64 [height][width][2] output: (R, Z) of the pixel's Ewald point
 *        S = (X/|X| - x)/lambda, X = (distance, y, z) (Eqs. laue, cyl-average), about the
 *        fibre axis n: Z = S_x sin(tilt) + S_z cos(tilt),
 *        R = sqrt((S_x cos(tilt) - S_z sin(tilt))^2 + S_y^2), binary64 without fused
 *        multiply-adds, sin and cos of the host's C library
 *   tile device float64 [n_tiles][8] output: R_lo, R_hi, Z_lo, Z_hi, P2_lo, P2_hi, 0, 0
 *        over the pixel centres of each tile, tiles row-major (fdtbx_tile_grid),
 *        n_tiles = tiles_x * tiles_y */
int fdtbx_pixel_map(const fdtbx_geometry* geom, double* pix, double* tile, void* stream);

/* Per-tile culling lists (under the mirror folds, of the launched tile columns and rows only;
 * the other tiles' lists are empty): reflection r is listed for tile t iff it is kept and
 *   R_lo(r) <= R_hi(t), R_lo(t) <= R_hi(r), Z_lo(r) <= Z_hi(t), Z_lo(t) <= Z_hi(r),
 *   P2_lo(r) <= P2_hi(t), P2_lo(t) <= P2_hi(r), and (if rho1 >= 0)
 *   max_corner(n1 . p) >= -rho1 and max_corner(n2 . p) >= -rho2 over the tile box corners,
 * in ascending reflection order.  Exact binary64 comparisons: reproducible bit for bit.
 *   offsets device int64 [n_tiles + 1] output (CSR row pointers)
 *   idx     device int32 [cap] output;  n_pairs host int64 output (total pairs)
 * Synchronises `stream` once to read the pair count.  If it exceeds cap,
 * returns FDTBX_ERR_BUFFER_TOO_SMALL with *n_pairs set and idx untouched.
 *   ws      device workspace of fdtbx_cull_workspace(geom, n_hkl) bytes
 * The tile grid is the one of fdtbx_pixel_map for geom. */
size_t fdtbx_cull_workspace(const fdtbx_geometry* geom, int64_t n_hkl);
int fdtbx_cull(const fdtbx_geometry* geom, const double* tile, int64_t n_hkl, const double* cull, int64_t* offsets,
               int32_t* idx, int64_t cap, int64_t* n_pairs, void* ws, size_t ws_bytes, void* stream);

/* Stacked tiles (the batched forward, fdtbx_batch_profile_stacked): the launched tile rows
 * taken two at a time, rows 2 sy and 2 sy + 1 forming stacked row sy (a single row last when
 * the launched rows are odd in number), so that one wave walks two tiles with one list.  The
 * grid of stacked tiles is tiles_x wide (fdtbx_tile_grid) and fdtbx_stacked_rows(geom) =
 * ceil(launched rows / 2) high, stacked tile s = sy tiles_x + sx.  Its box is the union of its
 * tiles' boxes, and its list is the culling list of fdtbx_cull for that box (the same
 * predicate), which contains the lists of both its tiles.
 *   fdtbx_stacked_rows   number of stacked rows (0 for an invalid geometry)
 *   fdtbx_stacked_boxes  stile device float64 [tiles_x * stacked rows][8] output, from the
 *                        tile boxes of fdtbx_pixel_map
 *   fdtbx_stacked_cull   as fdtbx_cull over the stacked grid (launched stacked columns only;
 *                        offsets [tiles_x * stacked rows + 1]), with the workspace of
 *                        fdtbx_stacked_cull_workspace; synchronises `stream` once */
int32_t fdtbx_stacked_rows(const fdtbx_geometry* geom);
int fdtbx_stacked_boxes(const fdtbx_geometry* geom, const double* tile, double* stile, void* stream);
size_t fdtbx_stacked_cull_workspace(const fdtbx_geometry* geom, int64_t n_hkl);
int fdtbx_stacked_cull(const fdtbx_geometry* geom, const double* stile, int64_t n_hkl, const double* cull,
                       int64_t* offsets, int32_t* idx, int64_t cap, int64_t* n_pairs, void* ws, size_t ws_bytes,
                       void* stream);

/* Launch order of the per-tile kernels (fdtbx_profile, fdtbx_profile_adjoint,
 * fdtbx_profile_cyl) for a set of culling lists: the tile each workgroup processes, -1 for
 * padding.  Workgroups are dealt to the 8 XCDs round-robin; tiles are grouped into
 * superblocks of 8 x 8 tiles (single tiles when the detector has fewer than 64
 * superblocks) that run on one XCD in consecutive dispatch slots.  When the launch holds
 * at most 8 rounds of workgroups per slot (16 per compute unit of the current device),
 * the superblocks run by decreasing length of their longest list and the tiles of a
 * superblock by decreasing list length (the long tiles start first); otherwise in index
 * order.  Performance only: every tile is listed once, and the images do not depend on
 * the order.
 *   offsets device int64 [n_tiles + 1] from fdtbx_cull
 *   order   device int32 [fdtbx_tile_order_size(geom)] output
 *   ws      device workspace of fdtbx_tile_order_workspace(geom) bytes */
int64_t fdtbx_tile_order_size(const fdtbx_geometry* geom);
size_t fdtbx_tile_order_workspace(const fdtbx_geometry* geom);
int fdtbx_tile_order(const fdtbx_geometry* geom, const int64_t* offsets, int32_t* order, void* ws, size_t ws_bytes,
                     void* stream);

/* The detector image (Eq. direct_sum per reflection at the pixel's query point
 * p* = R e_perp + Z z, Eq. lorentz):
 *   image[j][i] = delta/(R_ij + delta) * sum_hkl W_hkl r0^2 sum_k omega_k Z_hkl(p* - s_k)
 * with Z_hkl = prod_l f(N_l, a_l.(p* - s_k)), f the per-axis profile of the model's lineshape
 * (fdtbx_disorder), over nodes inside its support, reflections from the tile lists.
 *   order  device int32 [fdtbx_tile_order_size(geom)] from fdtbx_tile_order, or NULL (tiles
 *          in a fixed spatial order)
 *   image device float32 [height][width] output (fully overwritten)
 *   counts device int64 [1] (may be NULL): if non-NULL, a counting pass runs instead
 *          of the image pass and adds the number of (pixel, reflection, node) triples
 *          inside the support to *counts (image untouched). */
int fdtbx_profile(const fdtbx_model* model, const float* refl, const float* nodes, const double* pix,
                  const double* tile, const int64_t* offsets, const int32_t* idx, const int32_t* order, float* image,
                  int64_t* counts, void* stream);

/* fdtbx_profile_balanced: the image of fdtbx_profile (the same sum, Eqs. direct_sum and
 * lorentz) from a launch balanced over the compute units.  The launched tiles' lists are cut
 * into work units of geom.unit_pairs pairs (0: fdtbx_unit_pairs(n_pairs), read on the device
 * from offsets[n_tiles]); persistent waves take the units from eight queues, one per XCD
 * (slot b of the launch order feeds queue b % 8, in slot order), each unit writes its 64 pixel
 * sums to a slot of its own, and a second kernel adds each tile's units in unit order.  So no
 * long list runs as one workgroup at the end of the launch, and the image is the same on every
 * run; it equals fdtbx_profile's to float32 rounding (the sums are grouped by unit).
 *   order     as for fdtbx_profile (or NULL)
 *   pair_cap  capacity of idx: offsets[n_tiles] must not exceed it (units beyond the
 *             workspace's capacity, which only a larger total would need, are not run)
 *   ws        device workspace of fdtbx_profile_balanced_workspace(model, pair_cap) bytes:
 *             about 260 bytes per unit, for min(2^19, ceil(pair_cap / 32)) units plus one per
 *             tile when unit_pairs is 0 (at most 136 MB besides the tiles), ceil(pair_cap /
 *             unit_pairs) plus one per tile otherwise
 * fdtbx_unit_pairs(n): the library's pairs per unit for n culled pairs, max(32,
 * ceil(n / 2^19)) (0 for n < 0). */
int64_t fdtbx_unit_pairs(int64_t n_pairs);
size_t fdtbx_profile_balanced_workspace(const fdtbx_model* model, int64_t pair_cap);
int fdtbx_profile_balanced(const fdtbx_model* model, const float* refl, const float* nodes, const double* pix,
                           const double* tile, const int64_t* offsets, const int32_t* idx, const int32_t* order,
                           int64_t pair_cap, float* image, void* ws, size_t ws_bytes, void* stream);

/* Deterministic forward splat (the paper's projection path, sampled on a fixed grid
 * instead of at random; sections "Numerical evaluation: per-reflection shell quadrature",
 * "Lorentz correction on a sampled reciprocal lattice", "Analytical Solution of the Ewald
 * Diffraction Condition").  For each reflection h (fibre frame, radius r0, tangent frame
 * S0, e1, e2) and each sample
 *   r_a = r0 - dr + (a + 1/2) 2dr/n_r,  d_b = -Ts + (b + 1/2) 2Ts/n_s  (a < n_r; b < n_s per axis)
 *   S = (r c)((S0 + d1 e1) + d2 e2),  c = 1/sqrt((1 + d1^2) + d2^2)           (Eq. gnomonic)
 * with dr = sum_i w_i |a*_i| (w_i: the culling contract's support half-width bounds) and
 * Ts = min(T + 2 dr/r0, 10), the weight
 *   W_h I_h(S) delta/(R_S + delta) r^2 (2dr/n_r) c^3 (2Ts/n_s)^2,  I_h(S) = r0^2 sum_k omega_k Z(S - s_k)
 * is added to the pixels of both rotations about the fibre axis that put S on the Ewald
 * sphere (Eqs. harmonic, solutions; tilt as in fdtbx_geometry): S_x = -lambda |S|^2/2,
 * S.n = S_z(fibre), S_y = +-sqrt(|S|^2 - S_x^2 - S_z^2), k_out = (1/lambda + S_x, S_y, S_z),
 * pixel (floor(y/pixel + center_x), floor(z/pixel + center_y)) of y = distance k_y/k_x,
 * z = distance k_z/k_x (k_x > 0, on the detector).  Sample positions and pixels are
 * binary64 without fused multiply-adds, reproducible bit for bit; the weights are float32
 * accumulated with atomic adds (order-dependent in the last bits).
 *   hkl   device int32 [n_hkl][3]; refl, nodes: from fdtbx_reflection_prep, fdtbx_node_table
 *   n_r 1..1024, n_s 1..4096; n_hkl * n_r < 2^31
 *   image device float32 [height][width] output (zeroed by the call)
 *   counts device int64 [1] (may be NULL): if non-NULL, counts the (sample, node) pairs inside
 *          the support instead (image untouched). */
int fdtbx_splat(const fdtbx_model* model, const int32_t* hkl, int64_t n_hkl, const float* refl, const float* nodes,
                int32_t n_r, int32_t n_s, float* image, int64_t* counts, void* stream);

/* Exact cylindrical average (Eq. cyl-average) instead of the single-azimuth gather:
 *   image[j][i] = sum_h W_h (1/2 pi) sum_k dphi I_h(p_h(phi_k)),
 *   p_h(phi) = R cos(phi) e_perp + R sin(phi) e_az + Z z  (e_az = z x e_perp; (R, Z) of the pixel),
 * periodic trapezoid rule phi_k = k dphi, dphi = 2 pi/n, n = max(8, ceil(2 pi R/arc)),
 * k = -floor(n/2) .. ceil(n/2) - 1; no Lorentz factor (the ring average is the rotation
 * average).  I_h as in fdtbx_profile (lineshape included).
 *   offsets, idx: culling lists built by fdtbx_cull from fdtbx_cyl_records (the gather's lists
 *                 do not cover ring points off each reflection's azimuth)
 *   order: fdtbx_tile_order of those lists, or NULL (tiles in index order)
 *   arc: ring step, 1/A, in [1e-5, 1)
 *   image, counts: as in fdtbx_profile (counts: (pixel, ring point, node) triples) */
int fdtbx_profile_cyl(const fdtbx_model* model, const float* refl, const float* nodes, const double* pix,
                      const int64_t* offsets, const int32_t* idx, const int32_t* order, double arc, float* image,
                      int64_t* counts, void* stream);

/* Culling records (layout of fdtbx_reflection_prep's) for fdtbx_profile_cyl: with rho the
 * support corner radius sum_i w_i |a*_i| and rho_B = 2 r0 sqrt((1 - c_min)/2) + rho,
 * [0..3] = R_D -+ rho_B, D_z -+ rho_B, [4..5] = (max(r0 - rho, 0))^2, (r0 + rho)^2, wedge
 * disabled, [12] alive; binary64 +, -, *, /, sqrt only.
 *   cull device float64 [n_hkl][FDTBX_CULL_DOUBLES] output */
int fdtbx_cyl_records(const fdtbx_model* model, const int32_t* hkl, int64_t n_hkl, double* cull, void* stream);

/* ------------------------------------------------------------------ test-facing points */
/* The term of one reflection in the sum of Eq. direct_sum at arbitrary reciprocal points:
 *   out[k] = W_h r0^2 sum_nodes omega Z(p_k - s_node),  h = ridx[k],
 * i.e. the pattern's summand at p_k before the Lorentz factor (Eq. lorentz), with Z the
 * model's lineshape and the support test of fdtbx_profile.  One thread per point.
 *   hkl     device int32 [n_hkl][3] (the list refl was prepared from)
 *   refl    device float32 [n_hkl][FDTBX_REFL_FLOATS] (fdtbx_reflection_prep)
 *   nodes   device node table of the model (fdtbx_node_table)
 *   ridx    device int32 [n]: reflection of each point (index into hkl)
 *   points  device float64 [n][3]: Cartesian points of the laboratory frame, 1/A
 *   out     device float32 [n] output
 * n = 0 is valid (nothing is read or written). */
int fdtbx_profile_points(const fdtbx_model* model, const int32_t* hkl, const float* refl, const float* nodes,
                         const int32_t* ridx, const double* points, int64_t n, float* out, void* stream);

/* Forward Ewald projection (section "Analytical Solution of the Ewald Diffraction
 * Condition"): the detector positions of the two rotations about the (tilted) fibre axis n that
 * bring the point S onto the Ewald sphere (Eqs. harmonic, solutions).  S is given in the fibre
 * frame: S_z along n and (S_x, S_y) normal to it, so that only sqrt(S_x^2 + S_y^2) and S_z
 * matter (with no tilt this is the laboratory frame).  The projection is written
 * algebraically: the rotated S has S_x = -lambda |S|^2/2, S.n = Z_S and
 * S_y = +-sqrt(|S|^2 - S_x^2 - S_z^2); k_out = x/lambda + S meets the detector at
 * y = distance k_y/k_x, z = distance k_z/k_x.
 *   S    device float64 [n][3], 1/A
 *   out  device float64 [n][4]: (column, row) of the +S_y rotation, then of the -S_y one, as
 *        fractional pixel coordinates (pixel (i, j) covers [i, i+1) x [j, j+1)); all four NaN
 *        where no rotation satisfies the condition (Eq. valid) or k_x <= 0.
 * Binary64 without fused multiply-adds. */
int fdtbx_ewald_project(const fdtbx_geometry* geom, const double* S, int64_t n, double* out, void* stream);

/* ------------------------------------------------------------------ one-call pattern
 * fdtbx_profile_pattern runs reflection_prep, node_table, pixel_map, cull, tile_order
 * and the balanced profile launch (fdtbx_profile_balanced) into a caller workspace laid
 * out by fdtbx_pattern_workspace(model, n_hkl, pair_cap).  Synchronises once (pair count).  If the culling lists need
 * more than pair_cap entries it returns FDTBX_ERR_BUFFER_TOO_SMALL and writes
 * the required count to *pairs_needed (host, may be NULL); on success
 * *pairs_needed receives the pair count. */
size_t fdtbx_pattern_workspace(const fdtbx_model* model, int64_t n_hkl, int64_t pair_cap);
int fdtbx_profile_pattern(const fdtbx_model* model, const int32_t* hkl, int64_t n_hkl, const float* F2,
                          float* image, int64_t pair_cap, int64_t* pairs_needed, void* ws, size_t ws_bytes,
                          void* stream);

/* Device-written statistics of one fdtbx_profile_pattern_async call.  stamp[k] is the
 * device wall clock (clock_khz ticks per millisecond) when step k began: 0 reflection
 * preparation, 1 node table, 2 pixel map, 3 culling, 4 launch order, 5 profile, 6 counting
 * pass (when asked for), 7 the end; a step took (stamp[k+1] - stamp[k]) / clock_khz ms
 * (stamp[6] = stamp[7] without the counting pass). */
#define FDTBX_STATS_STAMPS 8
typedef struct fdtbx_stats {
  int64_t n_hkl;          /* reflections of the call */
  int64_t n_pairs;        /* (tile, reflection) pairs the culling lists need */
  int64_t pair_cap;       /* the capacity the call was given */
  int64_t useful_evals;   /* (pixel, reflection, node) triples inside the support, or -1 if not counted */
  int32_t overflow;       /* 1 if n_pairs > pair_cap: no lists were built and the image is all zero */
  int32_t n_stamps;       /* FDTBX_STATS_STAMPS */
  int64_t clock_khz;      /* rate of the stamps */
  uint64_t stamp[FDTBX_STATS_STAMPS];
} fdtbx_stats;

/* fdtbx_profile_pattern_async: fdtbx_profile_pattern without any host round trip, so that a
 * caller can capture it in a HIP graph: the pair capacity is checked on the device (with more
 * than pair_cap pairs the lists stay empty, the image comes out zero and stats->overflow is
 * set; the caller reads stats after the stream and retries with stats->n_pairs), every buffer
 * is cleared by a kernel, and nothing is copied to the host.  count_evals nonzero adds the
 * counting pass of fdtbx_profile (a second walk) for stats->useful_evals.
 *   stats  device fdtbx_stats [1] output (may be NULL)
 *   ws     device workspace of fdtbx_pattern_workspace(model, n_hkl, pair_cap) bytes, laid
 *          out as for fdtbx_profile_pattern, so fdtbx_pattern_backward can follow it. */
int fdtbx_profile_pattern_async(const fdtbx_model* model, const int32_t* hkl, int64_t n_hkl, const float* F2,
                                float* image, int64_t pair_cap, int32_t count_evals, fdtbx_stats* stats, void* ws,
                                size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------ adjoint
 * Gradients of a scalar L through the image, given G = dL/dimage (float32 [height][width],
 * device).  The parameters are the atoms (fractional x, y, z, B, occupancy) and the
 * FDTBX_N_GLOBALS globals; T stays fixed.  Profile values are recomputed tile by tile,
 * never stored.
 *
 * fdtbx_profile_adjoint: per reflection r, over the pixels of the tiles that list r and the
 * nodes inside the support (same lists, windows and kernel as fdtbx_profile), with
 * Z_k = C_r Z'_k the profile product of the lineshape and C_r = K_r/r0^2 the per-reflection
 * constant folded into the record:
 *   sums[r][0] = sum G L(R) sum_k omega_k Z'_k
 *   sums[r][1] = sum G L(R) sum_k (d omega_k/d sigma_theta) Z'_k
 *   sums[r][2] = sum G L(R) sum_k (d omega_k/d gamma_theta) Z'_k
 *   sums[r][3+i] = sum G L(R) sum_k omega_k N_i (dZ_k/dN_i)/C_r   (u held fixed)
 * sums: device float64 [n_hkl][6], zeroed by the call, then accumulated with binary64 atomic
 * adds (the result depends on the order of those adds only below binary64 rounding).
 * order: as in fdtbx_profile.
 * Under the up-down fold (bit 1 of geom.mirror) a computed pixel also stands for its mirror
 * (R, -Z), whose value reflection r gives through its Friedel mate: I_r(R, -Z) = I_{-r}(R, Z).
 * The kernel weights each pair's lane sums by G of the pixel (and its left-right mirror) into
 * r's sums and by G of the up-down mirrors into the sums of the mate -r, entry n_hkl - 1 - r of
 * the list (which must then be closed under negation in that order, as fdtbx_enumerate_hkl's
 * is), so the sums, dF2 and every gradient are those of the unfolded image, per reflection. */
int fdtbx_profile_adjoint(const fdtbx_model* model, const float* refl, const float* nodes, const double* pix,
                          const double* tile, const int64_t* offsets, const int32_t* idx, const int32_t* order,
                          int64_t n_hkl, const float* grad_image, double* sums, void* stream);

/* fdtbx_profile_adjoint_balanced: fdtbx_profile_adjoint over the work units of a
 * fdtbx_profile_balanced call (persistent waves taking the units from the eight XCD queues, so
 * no long list runs as one workgroup at the end).  bal_ws, bal_ws_bytes: the workspace of that
 * call, with the same model (unit_pairs included), lists, order and pair_cap, and no other
 * balanced launch on it since; its unit tables are read and its queue counters reused.  The
 * sums come out as fdtbx_profile_adjoint's (binary64 atomic adds, so their order and last bits
 * vary from run to run). */
int fdtbx_profile_adjoint_balanced(const fdtbx_model* model, const float* refl, const float* nodes, const double* pix,
                                   const double* tile, const int64_t* offsets, const int32_t* idx, const int32_t* order,
                                   int64_t pair_cap, int64_t n_hkl, const float* grad_image, double* sums, void* bal_ws,
                                   size_t bal_ws_bytes, void* stream);

/* Fixed-order (deterministic) accumulation of the same sums, in three calls (section
 * "Race detection" of the method's test strategy: gradients reproducible bit for bit).
 *
 * fdtbx_profile_adjoint_pairs: the walk of fdtbx_profile_adjoint, but pair p of the culling
 * lists (position p of idx) stores its twelve float32 lane-sum totals at partials[12 p]: the
 * six of its reflection r, then the six of the mate n_hkl - 1 - r (zero without the up-down
 * fold).  partials: device float32 [pair_cap][12], zeroed by the call (pairs that add nothing
 * keep zeros); pair_cap >= the pair count of the lists.
 *
 * fdtbx_pair_transpose: the pairs of each reflection in ascending list position, by a stable
 * radix sort of their reflection indices: refl_pairs[refl_ptr[r] .. refl_ptr[r+1]) are the
 * positions p with idx[p] = r.  n_pairs: device int64 [1] holding the pair count (for
 * instance offsets[n_tiles] of fdtbx_cull), or NULL when all pair_cap entries are pairs.
 *   refl_ptr   device int64 [n_hkl + 1] output;  refl_pairs device int32 [pair_cap] output
 *   ws         device workspace of fdtbx_pair_transpose_workspace(n_hkl, pair_cap) bytes
 *              (0 when pair_cap >= 2^31 or n_hkl >= 2^30: FDTBX_ERR_UNSUPPORTED)
 *
 * fdtbx_pair_reduce: sums[r][c] = sum over r's pairs p, in that order, of partials[p][c], plus
 * sum over the pairs p of its mate m of partials[p][6 + c], in binary64: m = mate[r] (device
 * int64 [n_hkl], -1 for none), or, with mate NULL, n_hkl - 1 - r if updown is nonzero and none
 * otherwise.  sums: device float64 [n_hkl][6] output.  No atomics: the same inputs give the
 * same bits on every run and every schedule. */
int fdtbx_profile_adjoint_pairs(const fdtbx_model* model, const float* refl, const float* nodes, const double* pix,
                                const double* tile, const int64_t* offsets, const int32_t* idx, const int32_t* order,
                                int64_t n_hkl, int64_t pair_cap, const float* grad_image, float* partials, void* stream);
size_t fdtbx_pair_transpose_workspace(int64_t n_hkl, int64_t pair_cap);
int fdtbx_pair_transpose(int64_t n_hkl, const int32_t* idx, int64_t pair_cap, const int64_t* n_pairs, int64_t* refl_ptr,
                         int32_t* refl_pairs, void* ws, size_t ws_bytes, void* stream);
int fdtbx_pair_reduce(int64_t n_hkl, const int64_t* refl_ptr, const int32_t* refl_pairs, const float* partials,
                      const int64_t* mate, int32_t updown, double* sums, void* stream);

/* fdtbx_adjoint_finish: chain rule per reflection in binary64 (Eqs. Ah, Neff, Ipara, axis
 * damping):
 *   dF2[r] = dL/d|F|^2 (device float32 [n_hkl] output, may be NULL)
 *   d_globals = dL/d(the FDTBX_N_GLOBALS globals) (device float64 [FDTBX_N_GLOBALS])
 * from the sums of fdtbx_profile_adjoint, the reflection records and F (device float32
 * [n_hkl][2]).  The globals are reduced over reflections in a fixed order.
 *   ws: device workspace of fdtbx_adjoint_finish_workspace(n_hkl) bytes */
size_t fdtbx_adjoint_finish_workspace(int64_t n_hkl);
int fdtbx_adjoint_finish(const fdtbx_model* model, const int32_t* hkl, int64_t n_hkl, const float* refl,
                         const double* sums, const float* F, float* dF2, double* d_globals, void* ws, size_t ws_bytes,
                         void* stream);

/* fdtbx_sf_adjoint: gradients of L through |F|^2 with respect to the atoms (Eq.
 * structure_factor): with t_j = occ_j f(s) exp(-B_j s^2) exp(2 pi i h.x_j),
 *   dL/dx_j = sum_r dF2_r 2 Re(F_r* 2 pi i h t_j)   (fractional x; y with k, z with l)
 *   dL/dB_j = sum_r dF2_r 2 Re(-s^2 F_r* t_j),  dL/docc_j = sum_r dF2_r 2 Re(F_r* t_j/occ_j)
 * Outputs device float32 [n_atoms] each (any may be NULL).  Deterministic (fixed-order
 * partial sums).  ws: device workspace of fdtbx_sf_adjoint_workspace(n_hkl, n_atoms) bytes. */
size_t fdtbx_sf_adjoint_workspace(int64_t n_hkl, int64_t n_atoms);
int fdtbx_sf_adjoint(const fdtbx_cell* cell, int64_t n_atoms, const float* x, const float* y, const float* z,
                     const float* B, const float* occ, const int32_t* type, const float* ff, int32_t n_types,
                     const int32_t* hkl, int64_t n_hkl, const float* F, const float* dF2, float* d_x, float* d_y,
                     float* d_z, float* d_B, float* d_occ, void* ws, size_t ws_bytes, void* stream);

/* fdtbx_pattern_backward: the three steps above after a successful fdtbx_profile_pattern
 * call with the same model, hkl, n_hkl and pair_cap, whose workspace fwd_ws still holds the
 * reflection records, node table, pixel map and culling lists.  F: the structure factors
 * whose |F|^2 the forward used.  Atom arrays as in fdtbx_structure_factors; gradient
 * outputs as in fdtbx_sf_adjoint (all five NULL skips the atom adjoint); d_globals as in
 * fdtbx_adjoint_finish; dF2 optional.  ws: device workspace of
 * fdtbx_backward_workspace(n_hkl, n_atoms) bytes. */
size_t fdtbx_backward_workspace(int64_t n_hkl, int64_t n_atoms);
int fdtbx_pattern_backward(const fdtbx_model* model, const int32_t* hkl, int64_t n_hkl, const float* F,
                           const float* grad_image, const void* fwd_ws, size_t fwd_ws_bytes, int64_t pair_cap,
                           int64_t n_atoms, const float* x, const float* y, const float* z, const float* B,
                           const float* occ, const int32_t* type, const float* ff, int32_t n_types, float* d_x,
                           float* d_y, float* d_z, float* d_B, float* d_occ, double* d_globals, float* dF2, void* ws,
                           size_t ws_bytes, void* stream);

/* fdtbx_pattern_backward_deterministic: fdtbx_pattern_backward with the fixed-order sums
 * (fdtbx_profile_adjoint_pairs, fdtbx_pair_transpose, fdtbx_pair_reduce) instead of atomic
 * adds: every output is reproducible bit for bit.  Same arguments; ws: device workspace of
 * fdtbx_backward_deterministic_workspace(n_hkl, n_atoms, pair_cap) bytes (about 60 bytes per
 * pair of capacity beyond fdtbx_backward_workspace; 0 for sizes the sort cannot take). */
size_t fdtbx_backward_deterministic_workspace(int64_t n_hkl, int64_t n_atoms, int64_t pair_cap);
int fdtbx_pattern_backward_deterministic(const fdtbx_model* model, const int32_t* hkl, int64_t n_hkl, const float* F,
                                         const float* grad_image, const void* fwd_ws, size_t fwd_ws_bytes,
                                         int64_t pair_cap, int64_t n_atoms, const float* x, const float* y,
                                         const float* z, const float* B, const float* occ, const int32_t* type,
                                         const float* ff, int32_t n_types, float* d_x, float* d_y, float* d_z, float* d_B,
                                         float* d_occ, double* d_globals, float* dF2, void* ws, size_t ws_bytes,
                                         void* stream);

/* fdtbx_pattern_backward_noalloc: fdtbx_pattern_backward for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  The same arguments without ws and ws_bytes: the workspace is a device array of
 * FDTBX_NOALLOC_SCRATCH_BYTES inside the library, one per device, held until the process
 * ends.  The call itself allocates nothing; the caller still passes the inputs, the forward
 * workspace and the outputs.  When fdtbx_backward_workspace(n_hkl, n_atoms) (n_atoms 0 when
 * the five atom outputs are NULL) exceeds the array it returns FDTBX_ERR_BUFFER_TOO_SMALL
 * before any launch (64 MiB covers the medium workload with its 5000 atoms, or about 1.3e6
 * reflections without atom gradients).  Every call on a device shares that device's array:
 * calls that overlap on one device (two streams, two threads) race and give wrong results;
 * calls in one stream's order are safe.  The array keeps the last call's contents, which no
 * later call reads before writing. */
#define FDTBX_NOALLOC_SCRATCH_BYTES (64u << 20)
int fdtbx_pattern_backward_noalloc(const fdtbx_model* model, const int32_t* hkl, int64_t n_hkl, const float* F,
                                   const float* grad_image, const void* fwd_ws, size_t fwd_ws_bytes, int64_t pair_cap,
                                   int64_t n_atoms, const float* x, const float* y, const float* z, const float* B,
                                   const float* occ, const int32_t* type, const float* ff, int32_t n_types, float* d_x,
                                   float* d_y, float* d_z, float* d_B, float* d_occ, double* d_globals, float* dF2,
                                   void* stream);

/* ------------------------------------------------------------------ batched models
 * Many models of different cells, atom counts, reflection lists and detectors in one
 * launch per step.  Each model's static data (reflection list, pixel map, tile boxes,
 * culling lists, scattering-factor table) is built beforehand with the single-model
 * entry points above and concatenated; fdtbx_batch_entry records where each model's
 * part starts.  Offsets count elements of the respective arrays (reflections, atoms,
 * pixels, tiles, CSR row pointers, culling-list entries, nodes, scattering-factor rows).
 * Every model keeps its own detector, quadrature and disorder parameters; the kernels
 * read them from the device copy of the entries, so the globals (sigma_theta, gamma_theta,
 * N_base, g, B_axis) can change between steps (fdtbx_batch_set_globals) without a host
 * round trip.  The
 * culling lists stay those built at set-up.
 *
 * Work tables (device int64, built by the caller): entries pack (model << 40) | first index.
 *   refl_blocks: blocks of 256 reflections, model-major (all blocks of a model adjacent);
 *   model_rb[n_models+1]: first refl_blocks entry of each model;
 *   atom_blocks: blocks of 256 atoms;  node_blocks: blocks of 256 node-table rows
 *               (fdtbx_node_rows(n_nodes) rows per model: node and block records);
 *   tile_items: (model, tile) pairs in the order the persistent kernels take them
 *               (longest culling list first balances the tail). */
typedef struct fdtbx_batch_entry {
  fdtbx_model model;
  double frame[19];     /* filled by fdtbx_batch_entry_init: rows a, b, c; rows a*, b*, c*; V */
  int64_t atom_off, n_atoms;
  int64_t hkl_off, n_hkl;
  int64_t pix_off;      /* first pixel of this model's image and pixel map */
  int64_t tile_off;     /* first tile box */
  int64_t rowptr_off;   /* first of this model's n_tiles + 1 CSR row pointers */
  int64_t pair_off;     /* first culling-list entry; the row pointers are relative to it */
  int64_t node_off;     /* first row of this model's node table (fdtbx_node_rows(n_nodes) rows) */
  int64_t ff_off;       /* first scattering-factor row */
  int32_t n_types, n_tiles;  /* scattering-factor rows (1..16) and tiles of this model */
  double setup_g[3];         /* g and N_base the culling lists were built with */
  double setup_N_base[3];
  int32_t stale;             /* set by fdtbx_batch_set_globals: 1 if the current globals widen a
                                support beyond those (some g_i > setup_g[i] or some
                                N_base_i < setup_N_base[i]), so the lists may miss pairs */
  int32_t reserved;
} fdtbx_batch_entry;

/* Host: validate the model and fill e->model, e->frame and e->setup_g, e->setup_N_base (from
 * the model: the parameters its culling lists are built with); offsets are the caller's. */
int fdtbx_batch_entry_init(const fdtbx_model* model, fdtbx_batch_entry* e);
/* Host: check host copies of the entries before they are uploaded: n_types in 1..16, sizes
 * and offsets non-negative.  FDTBX_ERR_INVALID_ARGUMENT names the first bad entry's field. */
int fdtbx_batch_entries_check(const fdtbx_batch_entry* entries, int32_t n_models);
/* sizeof(fdtbx_batch_entry), for bindings that mirror the struct. */
size_t fdtbx_batch_entry_size(void);

/* Device: entries[m].model.dis <- globals[m][0..FDTBX_N_GLOBALS-1] (order of FDTBX_N_GLOBALS),
 * and entries[m].stale <- whether those globals widen a lineshape support beyond the set-up
 * values (a larger g or a smaller N_base gives a smaller N_eff, hence a wider support in u; the
 * culling lists, built for the set-up supports, may then miss contributing pairs).  Smaller g,
 * larger N_base and every change of sigma_theta, gamma_theta and B_axis keep the lists exact
 * supersets.  (The reflection list keeps the set-up extinction cull: with g below its set-up
 * value a reflection it lacks has an intensity factor below exp(-limit (g/g_setup)^2).)
 * The caller reads the stale words back (outside any graph) before trusting the next step. */
int fdtbx_batch_set_globals(fdtbx_batch_entry* entries, int32_t n_models, const double* globals, void* stream);

/* Forward step for all models: structure factors F [sum n_hkl][2] and F2, reflection
 * records, node tables, and the images (float32, each [height][width] at pix_off).
 * counter: device int64 [2] scratch for the persistent kernel's work queue. */
int fdtbx_batch_forward(const fdtbx_batch_entry* entries, int32_t n_models, const int64_t* refl_blocks, int64_t n_rb,
                        const int64_t* node_blocks, int64_t n_nb, const int64_t* tile_items, int64_t n_items,
                        const int32_t* hkl, const float* x, const float* y, const float* z, const float* B,
                        const float* occ, const int32_t* type, const float* ff, const double* pix, const double* tile,
                        const int64_t* rowptr, const int32_t* idx, float* F, float* F2, float* refl, float* nodes,
                        float* image, int64_t* counter, void* stream);

/* The profile stage of fdtbx_batch_forward on stacked tiles (Eq. direct_sum at every pixel,
 * as fdtbx_batch_forward computes it): call fdtbx_batch_forward with n_items = 0 first (its
 * structure factors, records and node tables; no image), then this.  Each wave takes a
 * (model, stacked tile) item, packed (model << 40) | s, and walks the stacked tile's list once
 * for the pixels of both its tiles, so that the per-pair set-up and window scan are shared by
 * two tiles; every launched pixel of each item's tiles is written (with the mirror folds), so
 * the items must cover every launched stacked tile of every model.
 *   stack_off  device int64 [n_models][3]: the model's first stacked box in stile, first row
 *              pointer in srowptr and first list entry in sidx (row pointers relative to it)
 *   stile, srowptr, sidx  fdtbx_stacked_boxes and fdtbx_stacked_cull of each model, concatenated
 *   refl, nodes  as written by fdtbx_batch_forward; pix, tile as given to it
 *   counter    device int64 [2] scratch (the work queue)
 * The sums run in another grouping than the per-tile launch's, so the images agree with it to
 * float32 rounding.  Does not allocate, copy to the host or synchronise. */
int fdtbx_batch_profile_stacked(const fdtbx_batch_entry* entries, int32_t n_models, const int64_t* stack_off,
                                const int64_t* stack_items, int64_t n_items, const float* refl, const float* nodes,
                                const double* pix, const double* tile, const double* stile, const int64_t* srowptr,
                                const int32_t* sidx, float* image, int64_t* counter, void* stream);

/* Backward step for all models, after fdtbx_batch_forward with the same inputs:
 * grad_image (float32, laid out as the images) -> atom gradients (float32 [sum n_atoms]
 * each), d_globals (float64 [n_models][FDTBX_N_GLOBALS]) and dF2 (float32 [sum n_hkl]).  sums: device
 * float64 [n_hkl_total][6] scratch (n_hkl_total = sum of n_hkl); part: device float64
 * [n_rb][FDTBX_N_GLOBALS] scratch.  Neither call allocates, copies to the host or synchronises, so a
 * caller can capture them (with fdtbx_batch_set_globals) in a HIP graph. */
int fdtbx_batch_backward(const fdtbx_batch_entry* entries, int32_t n_models, const int64_t* refl_blocks, int64_t n_rb,
                         const int64_t* model_rb, const int64_t* atom_blocks, int64_t n_ab, const int64_t* tile_items,
                         int64_t n_items, int64_t n_hkl_total, const int32_t* hkl, const float* x, const float* y, const float* z,
                         const float* B, const float* occ, const int32_t* type, const float* ff, const double* pix,
                         const double* tile, const int64_t* rowptr, const int32_t* idx, const float* F,
                         const float* refl, const float* nodes, const float* grad_image, double* sums, double* part,
                         float* dF2, float* d_x, float* d_y, float* d_z, float* d_B, float* d_occ, double* d_globals,
                         int64_t* counter, void* stream);

/* fdtbx_batch_backward_deterministic: fdtbx_batch_backward with the fixed-order sums.
 * The batch's culling lists are fixed at set-up, so the caller builds, once, the order of
 * its pairs by reflection over the whole batch (global reflection index hkl_off + idx, global
 * pair index pair_off + position; as fdtbx_pair_transpose would): refl_ptr device int64
 * [n_hkl_total + 1], refl_pairs device int32 [n_pairs_total], and mate device int64
 * [n_hkl_total] (the global index of each reflection's Friedel mate, hkl_off + n_hkl - 1 - r,
 * for models with the up-down fold, else -1).  partials: device float32 [n_pairs_total][12]
 * scratch.  sums is then written by the reduction, not accumulated.  Graph-capturable like
 * fdtbx_batch_backward. */
int fdtbx_batch_backward_deterministic(
    const fdtbx_batch_entry* entries, int32_t n_models, const int64_t* refl_blocks, int64_t n_rb, const int64_t* model_rb,
    const int64_t* atom_blocks, int64_t n_ab, const int64_t* tile_items, int64_t n_items, int64_t n_hkl_total,
    const int32_t* hkl, const float* x, const float* y, const float* z, const float* B, const float* occ,
    const int32_t* type, const float* ff, const double* pix, const double* tile, const int64_t* rowptr, const int32_t* idx,
    const float* F, const float* refl, const float* nodes, const float* grad_image, int64_t n_pairs_total,
    const int64_t* refl_ptr, const int32_t* refl_pairs, const int64_t* mate, float* partials, double* sums, double* part,
    float* dF2, float* d_x, float* d_y, float* d_z, float* d_B, float* d_occ, double* d_globals, int64_t* counter,
    void* stream);

#ifdef __cplusplus
}
#endif
#endif /* FDTBX_H */
