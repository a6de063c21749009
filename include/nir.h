/*
 * nir.h - C ABI of the MI355X matrix-free spectral/hp operator library (libnir.so).
 *
 * The library evaluates the elemental operators of the spectral/hp element
 * method on batches ("blocks") of alike elements - hexahedra, prisms,
 * tetrahedra and pyramids with a modified C0 Jacobi basis - and composes them into the
 * Helmholtz operator H = L + lambda M.  The paper's statement of the problem
 * (section 3.1: a block of elements sharing shape, order, quadrature and a
 * deformed flag; operators that take basis/weight/derivative tensors and
 * produce a new block materialised into a caller's destination) is mirrored
 * by: a batch descriptor, library-owned basis tables, caller-owned geometry,
 * and distinct input and output buffers.
 *
 * Conventions shared by every call:
 *  - Pointers named "device" are device pointers (hipMalloc'd or torch CUDA
 *    tensors); pointers named "host" are ordinary host memory.  The caller
 *    owns every data array; the library owns only the opaque handles it
 *    creates (nir_basis, nir_mixed_plan, nir_cg_plan) and what they hold.
 *  - P is the number of modes per direction (polynomial order P-1), 2..10.
 *    Q is the number of quadrature points per direction; only Q = P+1 is
 *    supported by the kernels (NIR_ENOTSUP otherwise).
 *  - Modes of an element are stored contiguously, p outermost, r fastest,
 *    over the shape's mode set (hex p,q,r < P; prism r < P-p; tet q < P-p,
 *    r < P-p-q; pyramid r < P-max(p,q)): the packed order of the tet map,
 *    section 2.2 eq. (18), read lexicographically.  M = nir_nmodes(shape, P).
 *    The pyramid (no expansion in the paper) uses psi^a_p(eta1) psi^a_q(eta2)
 *    psi^b_{max(p,q),r}(eta3), both eta1 and eta2 collapsed at the apex, mode
 *    (0,0,1) being the apex function (1+eta3)/2; GLL points in eta1, eta2 and
 *    Gauss-Radau-Jacobi (alpha = 2) points in eta3.
 *  - Quadrature values are stored [elem][i][j][k], k fastest, npts = Q^3.
 *  - Geometry is stored SoA within an element: [elem][component][npts], or
 *    [elem][component] when the batch is not deformed (affine elements).
 *  - Every call validates its arguments on the host before any launch and
 *    returns NIR_EINVAL / NIR_ENOTSUP without touching the device; a failed
 *    launch returns NIR_EHIP.  nir_last_error() explains the last failure of
 *    the calling thread.  No C++ exception crosses the ABI.
 *  - Device work is enqueued on `stream` (a hipStream_t; NULL = the null
 *    stream) and is asynchronous; only nir_cg_solve and the *_create calls
 *    synchronise.  Inputs and outputs must not alias.
 *  - nelmt == 0 is valid and enqueues nothing.
 */
#ifndef NIR_H
#define NIR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NIR_OK = 0,
  NIR_EINVAL = 1,      /* invalid argument (null/misaligned pointer, bad size, aliasing) */
  NIR_ENOTSUP = 2,     /* valid but unsupported combination (e.g. Q != P+1) */
  NIR_ENOMEM = 3,      /* device or host allocation failed */
  NIR_EHIP = 4,        /* a HIP runtime call or kernel launch failed */
  NIR_ENONFINITE = 5,  /* NaN/Inf met in a solver input or iterate */
  NIR_EBREAKDOWN = 6,  /* CG breakdown (p^T A p <= 0) */
  NIR_ENOCONV = 7      /* iteration limit reached before the tolerance */
} nir_status;

typedef enum { NIR_HEX = 0, NIR_PRISM = 1, NIR_TET = 2, NIR_PYR = 3 } nir_shape;
typedef enum { NIR_F64 = 0, NIR_F32 = 1 } nir_dtype;               /* storage of coef/phys/geom */
typedef enum { NIR_MATH_NATIVE = 0, NIR_MATH_F16SPLIT = 1 } nir_math; /* contraction arithmetic */

/* A block of alike elements (paper section 3.1.1, the block type: shape,
 * basis/quadrature, Deformed flag, Size).  Enum-valued fields are int32_t
 * so that the layout is fixed. */
typedef struct {
  int32_t shape;     /* nir_shape */
  int32_t nmodes;    /* P, modes per direction, 2..10 */
  int32_t nquad;     /* Q, points per direction (must be P+1) */
  int32_t deformed;  /* 1: geometric factors per quadrature point; 0: per element */
  int64_t nelmt;     /* number of elements, >= 0 */
  int32_t dtype;     /* nir_dtype of coefficient, quadrature and geometry arrays */
  int32_t math;      /* nir_math: NIR_MATH_F16SPLIT only with NIR_F32 */
} nir_batch;

/* Number of modes per element: P^3 (hex), P^2(P+1)/2 (prism), P(P+1)(P+2)/6 (tet),
 * P(P+1)(2P+1)/6 (pyramid); -1 if invalid. */
int64_t nir_nmodes(int32_t shape, int32_t P);

/* Thread-local description of the last non-OK status returned on this thread. */
const char* nir_last_error(void);

/* Library version string. */
const char* nir_version(void);

/* ------------------------------------------------------------------ tables
 * 1-D quadrature on [-1,1] (host, no device needed).  rule 0: Gauss-Lobatto-
 * Legendre; rule 1: Gauss-Radau-Jacobi including x = -1 for the weight
 * (1-x)^alpha (alpha = 0, 1, 2).  Paper section 2.2 (collapsed directions
 * avoid the singular end point).  z, w: host arrays of Q doubles. */
nir_status nir_quadrature_host(int32_t rule, int32_t alpha, int32_t Q, double* z, double* w);

/* Identifiers of the per-(shape,P,Q) tables the kernels use (host copies via
 * nir_table_host).  Sizes in doubles (or int32 for the index tables):
 *  Z1,Z2,Z3 [Q]       points per direction (eta coordinates; eta = xi for the hex)
 *  W1,W2,W3 [Q]       weights per direction, collapse factors 1/2, 1/4 included
 *  T1,DT1   [P][Q]    direction-1 factor psi^a_p(eta_1i) and its derivative
 *  T2,DT2   [NP][Q]   direction-2 factor per (p,q) pair: psi^a_q (hex, prism) or psi^b_pq (tet)
 *  T3,DT3   [M][Q]    direction-3 factor per mode: psi^a_r, psi^b_pr (prism), psi^b_{p+q,r} (tet)
 *  D1,D2,D3 [Q][Q]    collocation derivative matrices D[i][l] = h_l'(z_i), section 2.2 eq. (22)
 *  WQ       [Q^3]     reference weight of each point (w1 w2 w3)
 *  XI       [3][Q^3]  reference coordinates xi of each point
 *  MODE_PQR [M][3]    int32: (p,q,r) of each mode                     (index table)
 *  POINT_IJK[Q^3][3]  int32: (i,j,k) of each point                    (index table)
 *  PAIR     [NP][4]   int32: (p, q, first mode m(p,q,0), count of r) of each (p,q) pair
 * NP = P^2 for hex and prism, P(P+1)/2 for the tet. */
typedef enum {
  NIR_TAB_Z1 = 0, NIR_TAB_Z2, NIR_TAB_Z3, NIR_TAB_W1, NIR_TAB_W2, NIR_TAB_W3,
  NIR_TAB_T1, NIR_TAB_DT1, NIR_TAB_T2, NIR_TAB_DT2, NIR_TAB_T3, NIR_TAB_DT3,
  NIR_TAB_D1, NIR_TAB_D2, NIR_TAB_D3, NIR_TAB_WQ, NIR_TAB_XI,
  NIR_TAB_MODE_PQR, NIR_TAB_POINT_IJK, NIR_TAB_PAIR, NIR_TAB_COUNT
} nir_table_id;

/* Number of elements of table `id` for (shape, P, Q); -1 if invalid. */
int64_t nir_table_size(int32_t shape, int32_t P, int32_t Q, int32_t id);

/* Copy table `id` into `out` (host; double* for FP tables, int32_t* for index tables;
 * `out` must hold nir_table_size() elements).  Host only, no device needed. */
nir_status nir_table_host(int32_t shape, int32_t P, int32_t Q, int32_t id, void* out);

/* Library-owned device copies of every table of (shape, P, Q) in FP64 and FP32. */
typedef struct nir_basis nir_basis;
nir_status nir_basis_create(int32_t shape, int32_t P, int32_t Q, nir_basis** out);
nir_status nir_basis_destroy(nir_basis* basis);
/* Device pointer of table `id` inside the handle (FP64, or int32 for index tables). */
const void* nir_basis_table_device(const nir_basis* basis, int32_t id);

/* ------------------------------------------------------------------ geometry
 * Caller-owned device geometry of a batch.  Paper section 2.1: W holds the
 * quadrature weight times det J (text after eq. (8)); PhysDeriv needs
 * d xi_j / d x_i at each point (eq. (9)).  npts = Q^3 if deformed, else 1.
 *   dxi_dx [nelmt][9][npts]  component 3a+i = d xi_a / d x_i
 *   jac    [nelmt][npts]     det J
 *   helm   [nelmt][7][npts]  fused Helmholtz factors: G_ab (ab = 00,01,02,11,12,22)
 *                            and Jw, with G_ab = Jw sum_i (d xi_a/d x_i)(d xi_b/d x_i),
 *                            Jw = det J * w_n (deformed) or det J (affine: the
 *                            kernels multiply by the point weight w_n).
 * Element type follows nir_batch.dtype.  Pointers not needed by a call may be NULL. */
typedef struct {
  const void* dxi_dx;
  const void* jac;
  const void* helm;
} nir_geom;

typedef enum { NIR_MAP_VERTEX = 0, NIR_MAP_VERTEX_SIN = 1 } nir_map;

/* FP64 geometric factors on the GPU from element vertices (device, [nelmt][nv][3]).
 * Reference vertices, in storage order:
 *   hex   (nv=8): (-1,-1,-1) (1,-1,-1) (1,1,-1) (-1,1,-1) (-1,-1,1) (1,-1,1) (1,1,1) (-1,1,1)
 *   prism (nv=6): (-1,-1,-1) (1,-1,-1) (1,1,-1) (-1,1,-1) (-1,-1,1) (-1,1,1)
 *   tet   (nv=4): (-1,-1,-1) (1,-1,-1) (-1,1,-1) (-1,-1,1)
 *   pyramid (nv=5): (-1,-1,-1) (1,-1,-1) (1,1,-1) (-1,1,-1) (-1,-1,1)  (base, then apex)
 * Map: trilinear hex / linear-triangle x linear prism / affine tet / the five pyramid vertex
 * functions (bilinear base times (1-xi3)/2 plus the apex function (1+xi3)/2; affine when the
 * base is a parallelogram) of the vertices; an affine batch (deformed = 0) evaluates its
 * constant Jacobian at the reference centroid; with
 * NIR_MAP_VERTEX_SIN every component is then moved by amp*sin(2 pi x)sin(2 pi y)sin(2 pi z).
 * Outputs (device, FP64, any may be NULL): dxi_dx, jac, helm64 with npts as above;
 * helm32 (FP32, optional) = round-to-nearest copy of helm64.  The batch dtype is
 * ignored (geometry is always computed in FP64).  det J is not checked on the device:
 * the caller's mesh must be orientation preserving at every quadrature point. */
nir_status nir_geom_from_vertices(const nir_batch* batch, const nir_basis* basis, const double* verts,
                                  int32_t map, double amp, double* dxi_dx, double* jac,
                                  double* helm64, float* helm32, void* stream);

/* FP64 geometric factors from caller-supplied Jacobians of the element map, for curved
 * elements whose map the library does not know (section 2.1: W is the point weight times det J,
 * and the physical derivative of eq. (9) needs d xi_j / d x_i; section 3.1.1: the block's
 * Deformed attribute selects factors per point or per element).
 *   jacobian [nelmt][9][npts] FP64 device array, component 3d+j = d x_d / d xi_j at point n
 *            (npts = Q^3 at the points of nir_table_host(NIR_TAB_XI) if batch->deformed, else 1:
 *            one constant Jacobian per affine element).
 * Outputs exactly as nir_geom_from_vertices (any may be NULL, not all): dxi_dx, jac, helm64 and
 * helm32 (the round-to-nearest FP32 copy), with the weights of the batch's quadrature.  The
 * batch dtype is ignored.  No output may overlap the Jacobians (NIR_EINVAL).  det J is not
 * checked on the device: a Jacobian that is singular or not orientation preserving gives
 * meaningless factors at that point. */
nir_status nir_geom_prepare(const nir_batch* batch, const nir_basis* basis, const double* jacobian, double* dxi_dx,
                            double* jac, double* helm64, float* helm32, void* stream);

/* Physical coordinates of the quadrature points (same maps as above): xyz [nelmt][3][Q^3]
 * FP64 device array.  Used to sample forcing functions at the points. */
nir_status nir_points_from_vertices(const nir_batch* batch, const nir_basis* basis, const double* verts,
                                   int32_t map, double amp, double* xyz, void* stream);

/* ------------------------------------------------------------------ operators
 * BwdTrans u = B u^ (section 2.2, eqs. (14)-(17)): coef [nelmt][M] -> phys [nelmt][Q^3]. */
nir_status nir_bwd_trans(const nir_batch* batch, const nir_basis* basis, const void* coef,
                         void* phys, void* stream);

/* PhysDeriv d_i = sum_j (d xi_j/d x_i) D_xi_j u (eq. (9), with the eta-to-xi chain rule
 * of eq. (23) for collapsed shapes): phys [nelmt][Q^3] -> d0, d1, d2 [nelmt][Q^3].
 * Uses geom->dxi_dx. */
nir_status nir_phys_deriv(const nir_batch* batch, const nir_basis* basis, const nir_geom* geom,
                          const void* phys, void* d0, void* d1, void* d2, void* stream);

/* IProductWRTBase u^ = B^T W f (eqs. (19)-(21)): phys [nelmt][Q^3] -> coef [nelmt][M].
 * Uses geom->jac (W = w_n det J). */
nir_status nir_iprod_wrt_base(const nir_batch* batch, const nir_basis* basis, const nir_geom* geom,
                              const void* phys, void* coef, void* stream);

/* IProductWRTDerivBase u^ = sum_i (D_{x_i} B)^T W f_i (the test_grad operation, section 3.1.2;
 * with eq. (7)): f0, f1, f2 [nelmt][Q^3] -> coef [nelmt][M].  Uses geom->dxi_dx and geom->jac. */
nir_status nir_iprod_wrt_deriv_base(const nir_batch* batch, const nir_basis* basis, const nir_geom* geom,
                                    const void* f0, const void* f1, const void* f2, void* coef,
                                    void* stream);

/* Fused Helmholtz y = (L + lambda M) u^ (section 2.1, eqs. (6), (7)) with every intermediate
 * on chip: coef_in [nelmt][M] -> coef_out [nelmt][M].  Uses geom->helm only.
 * batch->math = NIR_MATH_F16SPLIT (FP32 storage, hexahedra only; NIR_ENOTSUP otherwise) runs
 * the contractions as FP16 hi/lo split products on the matrix cores with FP32 accumulation.
 * The other operators accept NIR_MATH_NATIVE only. */
nir_status nir_helmholtz_apply(const nir_batch* batch, const nir_basis* basis, const nir_geom* geom,
                               double lambda, const void* coef_in, void* coef_out, void* stream);

/* Several fields per element (the block type's field count and its (fields, elements,
 * coefficients) layout permutation, section 3.1.1): y_f = (L + lambda M) u^_f for f < nfields,
 * every field of an element under that element's geometry.  coef_in and coef_out are
 * [nelmt][nfields][M] (fields interleaved per element), distinct and non-overlapping; geom as for
 * nir_helmholtz_apply (one set of factors per element, not per field).  The kernels run the
 * fields of an element in one workgroup, so its factors are read from HBM once.
 * nfields = 1 is nir_helmholtz_apply.  nfields = 2 or 3 needs hexahedra, Q = P + 1 and
 * NIR_MATH_NATIVE (FP64 or FP32); other field counts, shapes or math modes return NIR_ENOTSUP,
 * nfields < 1 NIR_EINVAL. */
nir_status nir_helmholtz_apply_fields(const nir_batch* batch, const nir_basis* basis, const nir_geom* geom,
                                      double lambda, int32_t nfields, const void* coef_in, void* coef_out,
                                      void* stream);

/* Trilinear hexahedra with the geometric factors formed in the kernel (section 2.1: they are the
 * metric terms of the element map at the points, and a trilinear map is fixed by its vertices):
 * y = (L + lambda M) u^ as nir_helmholtz_apply with the factors of
 * nir_geom_from_vertices(NIR_MAP_VERTEX), which are neither stored nor read.
 * verts: [nelmt][8][3] FP64 device array, vertex v at the reference corner
 * (s1, s2, s3) = (-,-,-), (+,-,-), (+,+,-), (-,+,-), then the same four at xi3 = +1 (the
 * order of nir_geom_from_vertices).  J, det J and the fused factors are computed in FP64 at
 * every point; FP32 batches round the factors to FP32 for the contractions.  Hexahedra,
 * Q = P + 1, NIR_MATH_NATIVE (else NIR_ENOTSUP); batch->deformed is not used; coef_in, coef_out
 * [nelmt][M], distinct; verts must not overlap coef_out.  A map that is not orientation
 * preserving at a point gives meaningless values there (not checked on the device). */
nir_status nir_helmholtz_apply_trilinear(const nir_batch* batch, const nir_basis* basis, const double* verts,
                                         double lambda, const void* coef_in, void* coef_out, void* stream);

/* The same weak operator (section 2.1, eqs. (6), (7)) in the nodal basis: the tensor-product
 * Lagrange polynomials through the Q = P + 1 GLL points of each direction (degree Q - 1), with
 * the values at those points as coefficients and the same points as quadrature (B = I, the
 * reference derivatives are the collocation matrices of nir_table_host(NIR_TAB_D1..3)):
 *   y = sum_a D_a^T (sum_b helm_ab D_b u) + lambda helm_6 u.
 * u_in, u_out: [nelmt][Q^3], point (i, j, k) at i Q^2 + j Q + k, distinct.  geom->helm exactly as
 * for nir_helmholtz_apply (the factors do not depend on the basis).  Hexahedra with Q = P + 1,
 * NIR_MATH_NATIVE (else NIR_ENOTSUP). */
nir_status nir_helmholtz_apply_nodal(const nir_batch* batch, const nir_basis* basis, const nir_geom* geom,
                                     double lambda, const void* u_in, void* u_out, void* stream);

/* ------------------------------------------------------------------ mixed batches
 * The fused Helmholtz apply over several batches of different shape and order (a mixed mesh
 * grouped by (shape, P)), replayed from one hipGraph.  Two strategies:
 *   NIR_MIXED_PERSISTENT  one persistent launch over a work list of element groups sorted by
 *                         decreasing cost; workgroup b of the grid of G runs items b, b+G, ...
 *                         with the group function of each item's (shape, P) (P <= 8: the
 *                         orders compiled into the persistent kernel);
 *   NIR_MIXED_PER_BATCH   one launch per batch with its standalone kernel (the variant selected
 *                         for its (shape, P, dtype) when the graph is captured), spread over
 *                         four parallel graph branches balanced by bytes;
 *   NIR_MIXED_AUTO        (default) the first apply times both and keeps the faster; plans
 *                         with a batch of P > 8 use NIR_MIXED_PER_BATCH.
 * Results of both equal the per-batch nir_helmholtz_apply launches (the same device code per
 * element group; bit for bit with the same kernel variant).  All batches share one dtype and
 * NIR_MATH_NATIVE; the arrays batches[], bases[], geoms[] (geoms[b].helm used) are copied, the
 * objects they point to must outlive the plan.  Tuning the persistent launch covers the
 * kernel's register budget (2..4 waves per SIMD) and the grid size (1..8 workgroups per CU),
 * timed on the caller's operands.  Changing the coefficient pointers or lambda between applies
 * re-uploads the descriptors (synchronising the stream) and re-captures a per-batch graph.
 * Not thread-safe per plan. */
typedef enum { NIR_MIXED_AUTO = 0, NIR_MIXED_PERSISTENT = 1, NIR_MIXED_PER_BATCH = 2 } nir_mixed_strategy;
typedef struct nir_mixed_plan nir_mixed_plan;
nir_status nir_mixed_plan_create(int32_t nbatch, const nir_batch* batches, const nir_basis* const* bases,
                                 const nir_geom* geoms, nir_mixed_plan** out);
/* coef_in[b], coef_out[b]: device arrays [nelmt_b][M_b] of batch b */
nir_status nir_mixed_helmholtz_apply(nir_mixed_plan* plan, double lambda, const void* const* coef_in,
                                     void* const* coef_out, void* stream);
/* Requests a strategy (nir_mixed_strategy); takes effect, with tuning, at the next apply.
 * NIR_ENOTSUP for NIR_MIXED_PERSISTENT on a plan with a batch of P > 8. */
nir_status nir_mixed_plan_set_strategy(nir_mixed_plan* plan, int32_t strategy);
/* Strategy in use (0 before the first apply) and the tuning times per apply (ms) of the two
 * strategies at the last tuning (-1 where not timed); any pointer may be NULL. */
nir_status nir_mixed_plan_timings(const nir_mixed_plan* plan, int32_t* strategy, double* ms_persistent,
                                  double* ms_per_batch);
/* work items of the persistent list, tuned grid size (0 before the first apply), the measured
 * time per apply (ms) of the strategy in use, algorithmic bytes and DoF of one apply; any
 * pointer may be NULL */
nir_status nir_mixed_plan_info(const nir_mixed_plan* plan, int32_t* nitems, int32_t* grid, double* tuned_ms,
                               int64_t* bytes, int64_t* dof);
nir_status nir_mixed_plan_destroy(nir_mixed_plan* plan);

/* Allocation-free persistent apply, for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, harnesses that forbid hipMalloc): one mixed apply over the
 * given batches with no plan.  It runs the persistent kernel of NIR_MIXED_PERSISTENT (register
 * budget of 2 waves per SIMD, one workgroup per CU per resident slot, no tuning), so each batch's
 * result equals nir_helmholtz_apply with the NIR_VARIANT_PENCIL kernel bit for bit.  Arguments
 * as nir_mixed_plan_create plus nir_mixed_helmholtz_apply; batches with nelmt = 0 are skipped.
 * lambda, the batch descriptors and the work list go to one static device array per GPU (about
 * 2.1 MB, held until the process ends), written by small kernels on `stream`; nothing is
 * allocated and the host arrays are read before the call returns.  Limits: nbatch <= 32, P <= 8,
 * at most 131072 work items (element groups of up to 32 elements, by shape and order),
 * NIR_EINVAL beyond them.  Every call on one GPU shares that array: calls that overlap on one GPU
 * (different streams or host threads without ordering) race and give wrong results. */
nir_status nir_mixed_helmholtz_apply_noalloc(int32_t nbatch, const nir_batch* batches, const nir_basis* const* bases,
                                             const nir_geom* geoms, double lambda, const void* const* coef_in,
                                             void* const* coef_out, void* stream);

/* ------------------------------------------------------------------ C0 assembly
 * Structured n x n x n hex mesh on a cube, element e = ix + n*(iy + n*iz), every element with
 * the same orientation (the paper leaves assembly out of scope, section 2.1).  The 1-D global
 * index of mode p of element i is i(P-1) + {0 if p = 0; P-1 if p = 1; p-1 if p >= 2}, and
 * the 3-D index is gz + ng*(gy + ng*gx), ng = n(P-1)+1 (z fastest, like r in the local mode
 * order, so gather and scatter read and write mostly contiguous runs); shared modes need no
 * sign change.
 * Number of global unknowns (n(P-1)+1)^3; -1 if invalid. */
int64_t nir_c0_nglobal_hex(int32_t n, int32_t P);
/* l2g [n^3][P^3] int32 local-to-global map: host version (host array) and device version
 * (device array, enqueued on stream).  NIR_EINVAL if the numbering exceeds int32. */
nir_status nir_c0_map_hex_host(int32_t n, int32_t P, int32_t* l2g);
nir_status nir_c0_map_hex(int32_t n, int32_t P, int32_t* l2g, void* stream);

/* Library-owned copy of a local-to-global map (device l2g [nelmt][M], values in [0, nglobal),
 * every global index used at least once) plus its inverse in CSR form, built on the host by a
 * stable counting sort: the entries of a global unknown are summed in ascending (element,
 * mode) order, so nir_scatter_add is deterministic.  Synchronous. */
typedef struct nir_assembly nir_assembly;
nir_status nir_assembly_create(const int32_t* l2g, int64_t nelmt, int32_t M, int64_t nglobal, nir_assembly** out);
nir_status nir_assembly_destroy(nir_assembly* a);
/* xl[e][m] = xg[l2g[e][m]]  (device arrays of `dtype`, xg [nglobal], xl [nelmt][M]) */
nir_status nir_gather(const nir_assembly* a, int32_t dtype, const void* xg, void* xl, void* stream);
/* yg[G] = sum of yl[e][m] over l2g[e][m] = G, fixed order (overwrites yg) */
nir_status nir_scatter_add(const nir_assembly* a, int32_t dtype, const void* yl, void* yg, void* stream);

/* Jacobi diagonal of the elemental Helmholtz operators: dl[e][m] = (H_e)_mm (device
 * [nelmt][M]); scatter-add gives the assembled diagonal.  Hex only (NIR_ENOTSUP otherwise).
 * Uses geom->helm. */
nir_status nir_helmholtz_diagonal(const nir_batch* batch, const nir_basis* basis, const nir_geom* geom,
                                  double lambda, void* dl, void* stream);

/* ------------------------------------------------------------------ CG solver
 * Jacobi-preconditioned CG on the assembled system A x = b, A = sum_e P_e^T H_e P_e (hex, FP64
 * batch).  The plan owns its workspace, a stream of its own (default priority) and the
 * hipGraphs that replay k = 10 PCG iterations with alpha/beta kept on the device; the host
 * reads the residual between graph launches.  Every solve is iterative refinement: the FP64
 * residual r = b - A x, an inner PCG on A d = r/||r||, and x += ||r|| d, until ||b - A x|| <=
 * rtol ||b||.  Modes:
 *   NIR_CG_FP64       inner PCG in FP64 run to the final tolerance (plain FP64 PCG)
 *   NIR_CG_MIXED_F32  inner PCG with FP32 vectors, FP32 element apply on the FP32 factors
 *                     (helm32 given at plan creation), FP64 dot products, stopped at inner_rtol
 *   NIR_CG_MIXED_F16SPLIT  as NIR_CG_MIXED_F32 with the element apply's contractions as
 *                     FP16-split products on the matrix cores (FP32 accumulation)
 * lambda may be any finite value; PCG needs A SPD (lambda > 0 with natural boundary
 * conditions), and an operator that is not reports NIR_EBREAKDOWN.
 * Errors: NIR_ENONFINITE (NaN/Inf in b or x0, or a non-finite residual), NIR_EBREAKDOWN
 * (FP64 p^T A p <= 0), NIR_ENOCONV (maxit inner iterations used; x and info still hold the
 * last iterate).  x holds x0 on entry (warm start / resume) and the solution on return.
 * Synchronous: returns after the solution is in x.  Not thread-safe per plan. */
typedef struct nir_cg_plan nir_cg_plan;
typedef enum { NIR_CG_FP64 = 0, NIR_CG_MIXED_F32 = 1, NIR_CG_MIXED_F16SPLIT = 2 } nir_cg_mode;
typedef struct {
  int32_t outer_iters;    /* refinement steps (FP64 residual evaluations after the first) */
  int32_t inner_iters;    /* PCG iterations over all inner solves */
  double rel_residual;    /* ||b - A x|| / ||b|| of the returned x, evaluated in FP64 */
  double seconds;         /* wall time of the solve */
} nir_cg_info;
nir_status nir_cg_plan_create(const nir_batch* batch64, const nir_basis* basis, const nir_geom* geom64,
                              const float* helm32, const nir_assembly* assembly, double lambda,
                              nir_cg_plan** out);
nir_status nir_cg_solve(nir_cg_plan* plan, int32_t mode, const double* b, double* x, double rtol, int32_t maxit,
                        double inner_rtol, nir_cg_info* info, void* stream);
nir_status nir_cg_plan_destroy(nir_cg_plan* plan);

/* ------------------------------------------------------------------ kernel variants and autotuning
 * Several kernels implement the fused Helmholtz apply (native contractions); the choice per
 * (shape, P, dtype) is library-global state (one int per combination, set atomically), used by
 * nir_helmholtz_apply and by the CG plans' element apply:
 *   NIR_VARIANT_AUTO       built-in default (a pencil kernel per shape; for hexahedra the
 *                          per-order choice measured fastest on MI355X)
 *   NIR_VARIANT_GENERIC    LDS-staged kernel, threads over points/modes (any shape)
 *   NIR_VARIANT_PENCIL     register-pencil kernel with uniform basis operands (any shape; on
 *                          prisms, tetrahedra and pyramids the contractions whose 1-D factor
 *                          depends on p, p+q or max(p,q) run one such index per wavefront)
 *   NIR_VARIANT_PENCIL_U2  hex pencil kernel with the streamed point loop unrolled twice
 *   NIR_VARIANT_PENCIL_E1  hex pencil kernel with one element per block (smaller LDS per block)
 *   NIR_VARIANT_PENCIL_PF  hex pencil kernel with each pencil's geometric factors loaded into
 *                          registers before the forward sweeps (latency overlap; for small P)
 *   NIR_VARIANT_PENCIL_SPLIT  hex pencil kernel whose planes between the direction-2 and
 *                          direction-1 sweeps pass through LDS two at a time (a third less LDS
 *                          per element, more blocks per CU at large P)
 *   NIR_VARIANT_PENCIL_GP  hex pencil kernel whose point loop requests the next point plane's
 *                          geometric factors while it computes the current one, the first plane
 *                          during the forward sweeps (deeper HBM latency overlap; per-point
 *                          factors only, otherwise the same as NIR_VARIANT_PENCIL)
 *   NIR_VARIANT_PENCIL_SPLIT_GP  the same on NIR_VARIANT_PENCIL_SPLIT (whose third plane then
 *                          stays in LDS during the point loop)
 *   NIR_VARIANT_PENCIL_EO  NIR_VARIANT_PENCIL_GP with every 1-D contraction folded over the
 *                          point pairs (i, Q-1-i) by the even-odd symmetry of the GLL points
 *                          and of the modified basis: about half the multiply-adds (results
 *                          differ from the unfolded kernels by rounding only)
 *   NIR_VARIANT_PENCIL_EO_SPLIT  the same on NIR_VARIANT_PENCIL_SPLIT_GP
 *                          (PF, GP, SPLIT_GP, EO and EO_SPLIT on per-point factors group a
 *                          per-order number of elements per block, measured on MI355X: as
 *                          few as one at large P, so that more, smaller blocks share a CU)
 *   NIR_VARIANT_DENSE      prisms, tetrahedra and pyramids with per-element factors (deformed = 0):
 *                          the operator as the seven reference matrices of the shape combined by
 *                          each element's factors, all elements of a launch stacked into one GEMM
 *                          on the FP64 or FP32 matrix cores (the reference matrices are
 *                          built with the generic kernel at nir_basis_create, for up to 256 modes
 *                          per element); other batches of these shapes run NIR_VARIANT_PENCIL.
 *                          The default for tetrahedra, prisms to P = 4 and pyramids to P = 6.
 * Setting a variant a shape does not support returns NIR_ENOTSUP. */
typedef enum { NIR_VARIANT_AUTO = 0, NIR_VARIANT_GENERIC = 1, NIR_VARIANT_PENCIL = 2,
               NIR_VARIANT_PENCIL_U2 = 3, NIR_VARIANT_PENCIL_E1 = 4, NIR_VARIANT_PENCIL_PF = 5,
               NIR_VARIANT_PENCIL_SPLIT = 6, NIR_VARIANT_PENCIL_GP = 7, NIR_VARIANT_PENCIL_SPLIT_GP = 8,
               NIR_VARIANT_PENCIL_EO = 9, NIR_VARIANT_PENCIL_EO_SPLIT = 10, NIR_VARIANT_DENSE = 11 } nir_variant;
nir_status nir_set_helmholtz_variant(int32_t shape, int32_t P, int32_t dtype, int32_t variant);
/* The variant a call with these parameters would run now (never NIR_VARIANT_AUTO); -1 if invalid. */
int32_t nir_get_helmholtz_variant(int32_t shape, int32_t P, int32_t dtype);
/* Autotuner: times every variant applicable to the batch's shape on the caller's operands
 * (one warm-up and `reps` timed applies each, hipEvents on `stream`; coef_out is overwritten),
 * selects the fastest for (shape, P, dtype) and returns it in *chosen.  ms_per_variant, if not
 * NULL, receives the average time of each variant at index variant-1 (11 doubles; untried
 * entries untouched).  Synchronises the stream. */
nir_status nir_autotune_helmholtz(const nir_batch* batch, const nir_basis* basis, const nir_geom* geom,
                                  double lambda, const void* coef_in, void* coef_out, int32_t reps,
                                  int32_t* chosen, double* ms_per_variant, void* stream);
/* JSON cache of the variant table: save writes every non-AUTO entry; load applies the entries of
 * a file written by save only if the whole file parses and validates (NIR_EINVAL otherwise, the
 * table unchanged).  Host only. */
nir_status nir_autotune_save(const char* path);
nir_status nir_autotune_load(const char* path);

#ifdef __cplusplus
}
#endif
#endif /* NIR_H */
