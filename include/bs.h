/*
 * bs.h -- C ABI of the Benchmark-Streaming operations for AMD Instinct MI355X
 * (gfx950).
 *
 * The seven streaming operations of a conjugate-gradient solve for high-order
 * hexahedral finite elements (Chalmers & Warburton, "Portable high-order
 * finite element kernels I: Streaming Operations", Table 1):
 *
 *   BS1 copy        y = x
 *   BS2 AXPY        y = alpha x + beta y
 *   BS3 norm        rho = x.x            (optionally weighted: sum w_i x_i^2)
 *   BS4 inner prod. sigma = x.y
 *   BS5 CG update   x += alpha p; r -= alpha Ap; rho = r.r   (Algorithm 1,
 *                   steps 8-10 fused)
 *   BS6 gather      x_G = Z^T x_L        (sum over local copies)
 *   BS7 scatter     x_L = Z x_G          (copy to local copies)
 *
 * plus the one-time mesh set-up that gather and scatter need (Section 5): the
 * scatter map Z of a structured hex mesh and the CSR form of Z^T.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Pointers named d_* and all vector arguments are DEVICE pointers on the
 *   context's device; the caller owns them.  The library owns only what it
 *   allocates inside bs_ctx and bs_gs objects.
 * - `stream` is a hipStream_t passed as void*; NULL means the null stream of
 *   the current device.  Every operation is asynchronous on that stream: it
 *   neither allocates, nor synchronises, nor reads back, so calls can be
 *   captured into a hipGraph.  The set-up calls (bs_ctx_create,
 *   bs_mesh_hex_map, bs_gs_create) allocate and synchronise.
 * - The calling thread's current HIP device must be the context's device.
 * - Lengths are int64_t; n == 0 is a valid no-op (reductions then write 0.0).
 * - Vectors must be aligned to their element size.  Writable vectors must
 *   not overlap any other argument; read-only inputs may alias each other
 *   (bs_dot(x, x) is fine).
 * - Reductions write one binary64 value to a caller-owned device double.
 *   Up to 128 workgroups a reduction finishes in the same launch (the last
 *   workgroup to publish its partial sum adds them all, in index order);
 *   longer grids take a second launch (Section 4 counts two launches for
 *   the paper's reductions).
 * - Arguments are validated on the host before anything is launched; a
 *   failed check returns BS_ERR_INVALID_ARG (or BS_ERR_UNSUPPORTED for a
 *   valid but unimplemented dtype) and launches nothing.  A HIP launch or
 *   runtime failure returns BS_ERR_HIP.  bs_last_error() then describes the
 *   failure of the calling thread's most recent unsuccessful call.
 * - One bs_ctx serves one stream at a time: its reduction workspace is
 *   reused by every reduction launched through it.
 * - Results are deterministic: the same inputs, sizes and context give the
 *   same bits on every call.
 */
#ifndef BS_H
#define BS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BS_F64 = 0,  /* binary64 storage and arithmetic                         */
  BS_F32 = 1,  /* binary32 storage, binary32 arithmetic                   */
  BS_BF16 = 2  /* bfloat16 storage, binary32 arithmetic                   */
} bs_dtype;

typedef enum {
  BS_OK = 0,
  BS_ERR_INVALID_ARG = 1,
  BS_ERR_UNSUPPORTED = 2,
  BS_ERR_ALLOC = 3,
  BS_ERR_HIP = 4,
  BS_ERR_NO_CONVERGENCE = 5
} bs_status;

typedef struct bs_ctx bs_ctx; /* per device: reduction workspace            */
typedef struct bs_gs bs_gs;   /* gather/scatter plan built from a map       */

/* Human-readable name of a status code (static storage). */
const char* bs_status_string(bs_status s);

/* Detail of the calling thread's most recent failure ("" if none). */
const char* bs_last_error(void);

/* Library version string (static storage). */
const char* bs_version(void);

/* Create a context on HIP device `device` (allocates its workspace, 33.6 MB
 * of reduction partials: one pair per workgroup for up to 2^21 workgroups,
 * plus 512 chunk sums; and synchronises).  *out receives the handle;
 * destroy it with bs_ctx_destroy. */
bs_status bs_ctx_create(int device, bs_ctx** out);
bs_status bs_ctx_destroy(bs_ctx* ctx);

/* Launch-shape knobs of one operation on this context (what the autotuner
 * sets).  op: 0 copy, 1 axpy, 2 norm, 3 dot, 4 cg_update, 5 gather,
 * 6 scatter, 7 batch (the persistent form of bs_batch_step: unroll is the
 * number of work items a workgroup claims per ticket, grid_cap caps the
 * workgroups below the resident count; variant unused; keyed by the
 * batch's number of work items).  unroll in {1, 2, 4, 8} is the number of 16-byte packets (or,
 * for scatter, entries) each thread handles per loop trip; grid_cap bounds
 * the number of workgroups (kernels grid-stride beyond it; reductions are
 * further capped at 2097152).  variant, for copy, axpy, norm, dot and
 * cg_update, is the workgroup order in its two low bits: 0 as the hardware
 * dispatches them (round-robin over the 8 XCDs, so the XCDs interleave 4 KB
 * slices of each operand), 1 the 256 workgroups one XCD receives in each
 * group of 2048 take consecutive block numbers (1 MB runs per XCD with
 * 256-thread workgroups), 2 each XCD takes one contiguous range of blocks
 * over the whole grid, 3 acts as 0; plus the workgroup size: + 4 for 128
 * threads, + 8 for 512 threads, otherwise 256 (operands not 16-byte aligned
 * with one another always run 256-thread workgroups); plus 16 for ordinary
 * cached loads and stores instead of nontemporal ones (faster when the
 * operands stay in the 256 MB last-level cache from one call to the next,
 * the small-size regime of Section 4's launch-latency model; calls whose
 * operands exceed 288 MiB run nontemporal whatever the variant).  For
 * gather and scatter, variant is a kernel choice,
 * plus 4 to keep the hardware's dispatch order or plus 8 for the runs of
 * 256 blocks per XCD in every group of 2048, instead of one contiguous range
 * of blocks per XCD, plus 16 for cached accesses in kernel 0 (as for the streaming
 * operations, with both value vectors and 4 bytes per local entry counted).  Gather: 0 = rows in the plan's permuted order (by default
 * in groups of 9 consecutive scatter tiles of the visiting order, each row
 * in the first group holding one of its copies, rows of a group in ascending
 * global id; bs_gs_order_rows and bs_gs_order_elements replace it; falls
 * back to 1 when a degree exceeds 1024), 1 = rows in global order, 2 = fixed blocks of 256 rows.  Scatter: 0 = tiles of 512 local
 * entries visited in order of their smallest global id, values read in
 * ascending global id and turned around in LDS, 1 = the same tiles read in
 * local order (for 0 and 1, `unroll` tiles per workgroup, at most 4),
 * 2 = local order with `unroll` entries per thread.  The setting applies to every dtype.  Results of the bit-exact
 * operations do not depend on it; reduction results depend on it only
 * through the order of their compensated additions.  Defaults: unroll 1
 * and one-pass grids for element-wise operations and gather/scatter;
 * norm and dot unroll 8 with 4096 workgroups; cg_update unroll 4 with
 * 65536 workgroups; gather and scatter variant 1 (a loaded tune table
 * replaces them, see below). */
bs_status bs_ctx_set_tune(bs_ctx* ctx, int op, bs_dtype dtype, int unroll, int grid_cap, int variant);

/* Tune entries by length.  Each (op, dtype) holds up to 16 entries; entry k
 * applies to lengths n >= n_min[k] up to the next entry (gather and scatter
 * look up the plan's local length).  bs_ctx_set_tune replaces them with one
 * entry for every dtype and length; bs_ctx_set_tune_entry inserts or
 * replaces the entry of one (op, dtype, n_min); bs_ctx_tune_for reports
 * the entry used for length n; bs_ctx_get_tune reports the n_min = 0 one;
 * bs_ctx_reset_tune restores what bs_ctx_create set up (the built-in
 * defaults, then the table beside the library or the one BS_TUNE_FILE
 * names; on a load error the defaults stay and the error is returned).
 *
 * bs_ctx_load_tune reads a text table, one entry per line:
 *     op dtype n_min unroll grid_cap variant      (# starts a comment)
 * with op in copy, axpy, norm, dot, cg_update, gather, scatter and dtype in
 * f64, f32, bf16.  Every (op, dtype) the table names gets exactly the
 * table's entries (which must include n_min 0); the others keep theirs.
 * Nothing is applied if any line is malformed (BS_ERR_INVALID_ARG, with the
 * line in bs_last_error).  *n_entries (may be NULL) gets the count.
 * bs_ctx_create loads the table that the environment variable BS_TUNE_FILE
 * names ("none": built-in defaults), else tune_gfx950.txt beside the
 * library if it exists (the autotuner's output), and fails if that table
 * is malformed. */
bs_status bs_ctx_set_tune_entry(bs_ctx* ctx, int op, bs_dtype dtype, int64_t n_min, int unroll, int grid_cap,
                                int variant);
bs_status bs_ctx_tune_for(const bs_ctx* ctx, int op, bs_dtype dtype, int64_t n, int* unroll, int* grid_cap,
                          int* variant);
bs_status bs_ctx_load_tune(bs_ctx* ctx, const char* path, int* n_entries);
bs_status bs_ctx_reset_tune(bs_ctx* ctx);
bs_status bs_ctx_get_tune(const bs_ctx* ctx, int op, bs_dtype dtype, int* unroll, int* grid_cap,
                          int* variant);

/* BS1 (Table 1; Listing 1): y[i] = x[i] for 0 <= i < n, bit for bit. */
bs_status bs_copy(bs_ctx* ctx, bs_dtype dtype, int64_t n, const void* x, void* y,
                  void* stream);

/* BS2 (Table 1; Listing 2): y[i] = alpha*x[i] + beta*y[i].
 * binary64: both products and the sum are rounded separately (no fused
 * multiply-add).  y is always read (beta == 0 does not skip it). */
bs_status bs_axpy(bs_ctx* ctx, bs_dtype dtype, int64_t n, double alpha, const void* x,
                  double beta, void* y, void* stream);

/* BS3 (Table 1; Listing 3): *d_out = sum_i w[i]*x[i]*x[i], the SQUARED norm
 * (no square root).  w == NULL means w[i] = 1, the paper's form; a non-NULL
 * w (for instance the 1/degree weights of bs_gs_weights) gives the weighted
 * inner product of the scattered form (Section 2).  Terms are rounded
 * products; the sum is compensated, so the result is within a few units in
 * the last place of the exact sum of the terms. */
bs_status bs_norm(bs_ctx* ctx, bs_dtype dtype, int64_t n, const void* x, const void* w,
                  double* d_out, void* stream);

/* BS4 (Table 1): *d_out = sum_i x[i]*y[i], accumulated with exact products
 * and compensated sums (accurate even for ill-conditioned sums). */
bs_status bs_dot(bs_ctx* ctx, bs_dtype dtype, int64_t n, const void* x, const void* y,
                 double* d_out, void* stream);

/* BS5 (Table 1; Algorithm 1 steps 8-10 fused, Section 3):
 *   x[i] <- x[i] + alpha*p[i];  r[i] <- r[i] - alpha*Ap[i];
 *   *d_rr = sum_i w[i]*r[i]*r[i] over the STORED updated r (w NULL => 1).
 * x and r are updated in place with separately rounded products and sums.
 * The CG ratio beta = rr_new/rr_old is left to the caller. */
bs_status bs_cg_update(bs_ctx* ctx, bs_dtype dtype, int64_t n, double alpha, void* x,
                       const void* p, void* r, const void* Ap, const void* w,
                       double* d_rr, void* stream);

/* Device-scalar forms of BS2 and BS5 for a CG iteration that stays on the
 * device (Algorithm 1, steps 7-11: alpha = r.r / p.Ap, the fused update,
 * beta = r'.r' / r.r and the direction update p = r + beta p), so that a
 * caller with an operator of its own can capture whole iterations into a
 * graph without reading a scalar back.  Each scalar is
 *     s = h * (num / den)
 * evaluated in binary64 as fl(h * fl(num / den)), where num = *d_num and
 * den = *d_den are device doubles read by the kernel when it starts (a
 * NULL pointer reads as 1.0, so with both NULL s = h), then rounded once to
 * the arithmetic type, exactly as bs_axpy / bs_cg_update round their host
 * scalars: with h = 1 and d_den = NULL the results equal those of the host
 * forms called with *d_num, bit for bit.  Division follows IEEE (den = 0
 * gives an infinity or NaN; the caller tests for breakdown).  The scalar
 * pointers must be 8-byte aligned; bs_cg_update_dev's d_rr must not be one
 * of them.  Otherwise as bs_axpy and bs_cg_update. */
bs_status bs_axpy_dev(bs_ctx* ctx, bs_dtype dtype, int64_t n, double alpha, const double* d_alpha_num,
                      const double* d_alpha_den, const void* x, double beta, const double* d_beta_num,
                      const double* d_beta_den, void* y, void* stream);
bs_status bs_cg_update_dev(bs_ctx* ctx, bs_dtype dtype, int64_t n, double alpha, const double* d_alpha_num,
                           const double* d_alpha_den, void* x, const void* p, void* r, const void* Ap,
                           const void* w, double* d_rr, void* stream);

/* BS5 for callers that cannot allocate device memory (code under graph
 * capture, serving loops, harnesses that forbid hipMalloc): the result of
 * bs_cg_update with no context.  The per-workgroup partial sums go to a
 * static device array of the library instead of a context's workspace:
 * 65,536 compensated pairs plus 16 chunk sums and a counter (1 MiB + 512 B
 * per device, held until the process ends), with the launch shape fixed at
 * 4 packets per thread and at most 65,536 workgroups, grid-striding over
 * longer vectors, so every length fits; a grid that would need more pairs is
 * rejected with BS_ERR_INVALID_ARG.  Nothing is allocated.  The pairs need
 * not start at zero (each call writes every pair it reads); the counter of
 * the single-launch finish (grids of at most 128 workgroups, as for the
 * context's reductions) starts at zero when the library loads and every
 * call that uses it leaves it at zero.  The
 * first call on a device looks the array's address up once (with that
 * device current).  Calls on one device share the array: calls that overlap
 * in time on one GPU (different streams, or threads) race and must be
 * serialised by the caller.  Results: x and r bit-identical to bs_cg_update;
 * *d_rr equal to bs_cg_update's under the same launch shape (its built-in
 * shape for the CG update) and within 1e-14 of the exact sum otherwise.
 * Arguments, validation and aliasing rules as bs_cg_update; the vectors and
 * d_rr must be on the current device. */
bs_status bs_cg_update_noalloc(bs_dtype dtype, int64_t n, double alpha, void* x, const void* p, void* r,
                               const void* Ap, const void* w, double* d_rr, void* stream);

/* Scatter map of a structured K x K x K hex mesh of degree N (Section 2,
 * eq. scatter_def): for element slot s (0 <= s < K^3) and local node
 * (i,j,k) (0 <= i,j,k <= N), local index l = s*(N+1)^3 + i + (N+1)*(j + (N+1)*k)
 * gets the global id X + M*(Y + M*Z), M = K*N+1, of its lattice point.
 * Slot s holds lattice element e = d_perm[s] at (e%K, (e/K)%K, e/K^2),
 * turned by orientation d_orient[s] in [0,24): a permutation pi of the axes
 * (lexicographic order) and flip bits f0+2f1+4f2, keeping the 24 proper
 * rotations in that order (0 is the identity); local (i,j,k) = t lands on
 * lattice offset o_d = t[pi[d]], or N - t[pi[d]] when flip d is set.
 * d_perm (int32[K^3]) and d_orient (uint8[K^3]) may be NULL for the
 * lexicographic, unrotated mesh.  d_map is int32[K^3 (N+1)^3].
 * Requires (K*N+1)^3 < 2^31 and K^3 (N+1)^3 < 2^31.  Synchronises `stream`;
 * returns BS_ERR_INVALID_ARG if a perm entry lies outside [0, K^3) or an
 * orientation outside [0, 24). */
bs_status bs_mesh_hex_map(int64_t K, int N, const int32_t* d_perm, const uint8_t* d_orient,
                          int32_t* d_map, void* stream);

/* The same map computed on the host into host memory (same arguments, host
 * pointers; perm/orient may be NULL). */
bs_status bs_mesh_hex_map_host(int64_t K, int N, const int32_t* perm, const uint8_t* orient,
                               int32_t* map);

/* Build a gather/scatter plan from a scatter map d_map[n_local] (Section 5):
 * entries in [0, n_global) are global ids, negative entries are masked
 * (excluded from gather, untouched by scatter).  The plan keeps its own copy
 * of the map and builds the CSR form of Z^T without values: row g lists the
 * unmasked local indices l with map[l] == g in ascending order.  Requires
 * n_local, n_global < 2^31.  Allocates and synchronises `stream`; returns
 * BS_ERR_INVALID_ARG if any entry is >= n_global. */
bs_status bs_gs_create(bs_ctx* ctx, const int32_t* d_map, int64_t n_local, int64_t n_global,
                       void* stream, bs_gs** out);
bs_status bs_gs_destroy(bs_gs* gs);

/* Replace the plan's permuted row order (gather kernel 0: variants 0, 4, 8)
 * and its scatter tile order with ones grouped by elements (Section 5: each
 * workgroup of the gather sums the rows of a few neighbouring elements, so
 * that their local values are read while in cache).  Elements are the
 * n_local / nodes_per_element runs of consecutive local indices (as in
 * Listings 4 and 5, local index e * nodes_per_element + node).  Elements are
 * visited in groups of elements_per_group consecutive visiting ranks; each
 * row is keyed by the smallest group of an element holding one of its
 * copies, and the rows of one group stay in ascending global id (so that a
 * workgroup writes x_G in runs wherever the global numbering has them).
 * d_elem_rank (device int32[n_elem], values in [0, 2^31)) gives the visiting
 * ranks; when it is NULL the library derives them from the map alone:
 * elements sharing a face are neighbours, and the element graph is ordered
 * by recursive bisection at the median of breadth-first distances from a
 * far element of each part (no coordinates and no numbering of the global
 * ids are used).  That form needs nodes_per_element = (N+1)^3, N >= 1, with
 * the local node numbering of bs_mesh_hex_map, copies the 8 n_elem corner
 * ids to the host and takes host time roughly linear in n_elem (seconds at
 * 2 million elements).  The scatter (bs_gs_scatter) visits its tiles in the
 * same groups.  Gather and scatter results are the same bits in every
 * order.  Allocates and synchronises `stream`; BS_ERR_INVALID_ARG if
 * n_local is not a multiple of nodes_per_element or elements_per_group < 1. */
bs_status bs_gs_order_elements(bs_gs* gs, int64_t nodes_per_element, const int32_t* d_elem_rank,
                               int64_t elements_per_group, void* stream);

/* Replace the plan's permuted row order (gather kernel 0: variants 0, 4, 8) with a
 * lattice-tiled one, for maps whose global ids are lattice points
 * g = X + mx (Y + my Z) (mx*my*mz == n_global): rows in tile x tile x tile
 * blocks of the lattice, blocks in lattice order (x fastest); inside a
 * block, rows in bx x by x bz boxes, boxes in lattice order (a side of 0,
 * or above tile, is the tile's: 0, 0, 0 is one box); ascending g within a
 * box; rows without copies last.  Boxes matched to the elements in y and z
 * (sides a multiple of the degree N on the meshes of bs_mesh_hex_map, with
 * tile a multiple of them) let a gather workgroup read longer runs of each
 * element's local values; the tiles keep the elements around a tile in
 * cache while all their copies are added.  The result is the same (each
 * row is still summed in ascending local index).  Allocates and
 * synchronises `stream`; BS_ERR_INVALID_ARG for a negative side or more
 * than 2^32 - 1 boxes, BS_ERR_UNSUPPORTED when the plan has no permuted
 * order (a degree above 1024); on failure the previous order stays in
 * place. */
bs_status bs_gs_order_rows(bs_gs* gs, int64_t mx, int64_t my, int64_t mz, int32_t tile, int32_t bx, int32_t by,
                           int32_t bz, void* stream);

/* Sizes of a plan: local length, global length, unmasked local entries,
 * largest node degree.  Any output pointer may be NULL. */
bs_status bs_gs_info(const bs_gs* gs, int64_t* n_local, int64_t* n_global,
                     int64_t* n_unmasked, int64_t* max_degree);

/* Copy the plan's CSR arrays into caller buffers: d_row_starts int32[n_global+1],
 * d_col_ids int32[n_unmasked]. */
bs_status bs_gs_csr(const bs_gs* gs, int32_t* d_row_starts, int32_t* d_col_ids, void* stream);

/* d_deg[g] = number of unmasked local copies of global node g (int32[n_global]). */
bs_status bs_gs_degree(const bs_gs* gs, int32_t* d_deg, void* stream);

/* d_wL[l] = 1/deg(map[l]) (correctly rounded division) for unmasked l,
 * 0 for masked l; d_wL has n_local entries of `dtype`. */
bs_status bs_gs_weights(const bs_gs* gs, bs_dtype dtype, void* d_wL, void* stream);

/* BS6 (Table 1; Listing 4): x_G[g] = sum of x_L[l] over row g of the CSR,
 * added one at a time in ascending l starting from +0.0; rows with no copies
 * give +0.0.  x_L has n_local entries, x_G n_global. */
bs_status bs_gather(bs_ctx* ctx, const bs_gs* gs, bs_dtype dtype, const void* xL, void* xG,
                    void* stream);

/* BS7 (Table 1; Listing 5; eq. scatter_def): x_L[l] = x_G[d_map[l]] for
 * 0 <= l < n_local where 0 <= d_map[l] < n_global; other entries of x_L are
 * left untouched (negative ids are masked, as in Listing 5; ids >= n_global
 * are treated the same way, so a bad id never reads outside x_G).  d_map
 * (int32[n_local], device) is read directly, as the listing's scatterIds:
 * no plan is needed.  Bit-exact copy of the values.  x_L must not overlap
 * x_G or d_map.  The tune entry of the scatter (op 6) gives the entries per
 * thread (unroll) and the grid cap. */
bs_status bs_scatter(bs_ctx* ctx, bs_dtype dtype, int64_t n_local, const int32_t* d_map, int64_t n_global,
                     const void* xG, void* xL, void* stream);

/* BS7 through a plan (Table 1; Listing 5; Section 5): the same result as
 * bs_scatter with the plan's map, by the kernel the tune entry selects
 * (sorted tiles visited in order of their smallest global id, by default).
 * The plan's map was validated when the plan was built. */
bs_status bs_gs_scatter(bs_ctx* ctx, const bs_gs* gs, bs_dtype dtype, const void* xG, void* xL,
                        void* stream);

/* ---------------------------------------------------------------------------
 * Element operators of the Helmholtz problem inside the scattered form
 * (Section 2, eqs. helm_var, global_system, assembled_stiff, assembled_mass):
 * y_G = Z^T A_L Z x_G with A_L block diagonal, binary64.
 *
 * Basis: tensor-product Lagrange polynomials through the N+1 Gauss-Lobatto-
 * Legendre (GLL) points per axis, local node i + (N+1)(j + (N+1) k) as in
 * bs_mesh_hex_map.  Element integrals use the N+1 point Gauss-Legendre rule
 * (exact for products of degree-N polynomials) on affine hexahedra, whose
 * geometry is given per element e as seven doubles
 *     d_geo[7e .. 7e+6] = (G11, G12, G13, G22, G23, G33, |J|),
 * G = |J| J^-1 J^-T (for an axis-aligned cube of side h in any orientation,
 * G = (h/2) I and |J| = (h/2)^3).  Then
 *     A^e = S^e + lambda M^e,  S^e = sum_dd' A_d^T W G_dd' A_d',
 *     M^e = |J| Bq^T W Bq,
 * A_1 = B x B x D (derivative along i), A_2 = B x D x B, A_3 = D x B x B,
 * B[a][i] = l_i(xi_a), D[a][i] = l_i'(xi_a) at the Gauss points xi_a,
 * W the product Gauss weights.  The lumped mass puts the GLL rule on the
 * nodes: the diagonal block d_l = |J| w_i w_j w_k (GLL weights).
 * ------------------------------------------------------------------------- */

typedef struct bs_elem bs_elem; /* the 1D rules and basis tables of degree N */

/* Rules and basis tables of degree N in [1, 15] on the context's device
 * (the local Helmholtz operator supports N <= 7; the lumped mass any N).
 * Nodes and weights come from Newton iterations in extended precision,
 * rounded to binary64.  Allocates and synchronises. */
bs_status bs_elem_create(bs_ctx* ctx, int N, bs_elem** out);
bs_status bs_elem_destroy(bs_elem* el);

/* Host copies of the rules (N+1 values each; any pointer may be NULL):
 * GLL nodes and weights, Gauss-Legendre nodes and weights, ascending. */
bs_status bs_elem_rules(const bs_elem* el, double* gll_x, double* gll_w, double* gauss_x, double* gauss_w);

/* y_L = A_L Z x_G for n_elem elements whose local nodes are numbered
 * e (N+1)^3 + i + (N+1)(j + (N+1) k): each element's values are read
 * through d_map[n_elem (N+1)^3] from x_G (ids outside [0, n_global) read
 * 0, as for masked nodes) and never stored as x_L (the scatter is fused
 * into the operator); y_L (binary64[n_elem (N+1)^3]) receives A^e u^e.
 * Sum-factorised on the matrix cores (MFMA); the result equals the dense
 * blocks' product up to rounding (it is not bit-reproducible against a
 * different evaluation order).  BS_ERR_UNSUPPORTED for N > 7.  y_L must
 * not overlap the inputs.  Asynchronous. */
bs_status bs_helmholtz_local(bs_ctx* ctx, const bs_elem* el, int64_t n_elem, const int32_t* d_map,
                             int64_t n_global, const double* d_geo, double lambda, const double* xG, double* yL,
                             void* stream);

/* y_G = Z^T A_L Z x_G on a plan: bs_helmholtz_local with the plan's map
 * into the caller's work vector yL_work (binary64[n_local]), then the
 * gather (BS6) of yL_work into y_G.  Asynchronous. */
bs_status bs_helmholtz_apply(bs_ctx* ctx, const bs_elem* el, const bs_gs* gs, const double* d_geo, double lambda,
                             const double* xG, double* yL_work, double* yG, void* stream);

/* Lumped mass y_G = Z^T D_L Z x_G without a local vector: y_G[g] adds
 * fl(d_l x_G[g]) over the copies l of g in ascending l from +0.0 (the
 * gather's order, Listing 4), d_l = fl(fl(fl(w_i w_j) w_k) |J_e|) computed
 * from the column's element e and node (i, j, k).  One pass over the CSR
 * of Z^T: reads x_G once, writes y_G once.  Asynchronous. */
bs_status bs_mass_lumped(bs_ctx* ctx, const bs_elem* el, const bs_gs* gs, const double* d_geo, const double* xG,
                         double* yG, void* stream);

/* ---------------------------------------------------------------------------
 * Conjugate gradients built from the operations above (Algorithm 1), on the
 * 7-point finite-difference operator
 *   (A x)_ijk = (6 + shift) x_ijk - x_(i-1)jk - x_(i+1)jk - x_i(j-1)k
 *               - x_i(j+1)k - x_ij(k-1) - x_ij(k+1)
 * on an m x m x m grid of unknowns, index i + m*(j + m*k), with zero
 * Dirichlet ghost values.  The additions run in exactly that order (absent
 * neighbours skipped), with 6 + shift computed in binary64 and rounded once
 * to the working precision, so the binary64 operator is reproducible bit
 * for bit.
 * ------------------------------------------------------------------------- */

/* y = A x on the m^3 grid (x, y of `dtype`, m^3 entries each; binary32
 * arithmetic for the narrow dtypes).  Asynchronous like the seven ops. */
bs_status bs_stencil7(bs_ctx* ctx, bs_dtype dtype, int64_t m, double shift, const void* x, void* y,
                      void* stream);

typedef struct {
  int64_t iterations;       /* CG iterations (all inner iterations for IR)       */
  int64_t outer_iterations; /* refinement steps (0 for bs_cg_solve)              */
  int64_t restarts;         /* restarts from the true residual (bs_cg_solve)     */
  double rel_residual;      /* ||b - A x||_2 / ||b||_2 at exit, binary64, true   */
  double seconds;           /* wall time of the call                             */
} bs_cg_result;

/* Solve A x = b in binary64 by CG, starting from the given x (d_b, d_x:
 * binary64[m^3] device vectors; x is overwritten).  Stops when the true
 * relative residual ||b - Ax|| / ||b|| <= tol (iteration stops on the
 * recursive residual r.r first, then the true residual is recomputed and CG
 * restarts from it if needed), or after max_iter iterations in total.  The
 * scalars of each iteration stay on the device and batches of iterations
 * run as one captured HIP graph.  Allocates its workspace (3 vectors) and
 * synchronises `stream`; returns BS_ERR_NO_CONVERGENCE if tol is not met.
 * m^3 must stay below 2^31. */
bs_status bs_cg_solve(bs_ctx* ctx, int64_t m, double shift, const double* d_b, double* d_x, double tol,
                      int64_t max_iter, bs_cg_result* res, void* stream);

/* Mixed-precision iterative refinement: binary64 residual r = b - A x,
 * ||r|| and update x += ||r|| d; the correction d solves A d = r/||r|| by CG
 * with vectors stored in `inner` (BS_F32 or BS_BF16; BS_F64 is accepted)
 * and binary32 arithmetic, to relative residual inner_tol (or the looser
 * 0.5 tol ||b|| / ||r|| when that already meets the outer target) or
 * max_inner iterations.  Stops when the true relative residual <= tol, after
 * max_outer refinement steps, or when the outer residual fails to halve over
 * three steps (BS_ERR_NO_CONVERGENCE, with res still filled in).  x starts
 * from its given value.  Allocates its workspace and synchronises `stream`. */
bs_status bs_cg_ir_solve(bs_ctx* ctx, bs_dtype inner, int64_t m, double shift, const double* d_b, double* d_x,
                         double tol, double inner_tol, int64_t max_inner, int64_t max_outer, bs_cg_result* res,
                         void* stream);

/* Solve (S + lambda M) x = b by CG (Algorithm 1) in binary64, where
 * S + lambda M = Z^T A_L Z is the assembled Helmholtz operator of
 * bs_helmholtz_apply (Section 2, eqs. global_system, assembled_stiff,
 * assembled_mass): gs is the plan of the scatter map (masked copies are
 * Dirichlet nodes, left out of Z), el the degree (N <= 7), d_geo the
 * per-element factors as for bs_helmholtz_local.  d_b, d_x: binary64
 * [n_global] device vectors; x is the starting guess and is overwritten; x
 * must not overlap b.  The operator must be positive definite on the
 * unmasked nodes (lambda > 0, or a stiffness with enough masked nodes).
 * Stopping, restarts and the result record as for bs_cg_solve.  Each
 * iteration: the local operator on p (the scatter fused into its load) with
 * the partial sums of p.Ap formed there (the sum over elements of
 * u_e . A^e u_e, equal to p . Z^T A_L Z p), the gather (Listing 4), alpha,
 * the update (BS5), beta and the direction (BS2), the scalars on the
 * device; batches of iterations run as one captured HIP graph.  Allocates
 * its workspace (3 global vectors and one local vector), synchronises
 * `stream`; BS_ERR_NO_CONVERGENCE if tol is not met within max_iter. */
bs_status bs_helmholtz_cg_solve(bs_ctx* ctx, const bs_elem* el, const bs_gs* gs, const double* d_geo, double lambda,
                                const double* d_b, double* d_x, double tol, int64_t max_iter, bs_cg_result* res,
                                void* stream);

/* ---------------------------------------------------------------- batched instances
 *
 * Many independent instances of uneven size run as one batch (the launch
 * latency + bandwidth model of Section 4: short vectors are dominated by the
 * per-launch cost, so they are processed together).  Instance i has global
 * vectors of n_global[i] entries and local vectors of n_local[i] entries;
 * every vector argument is the concatenation of all instances' vectors in
 * instance order (offsets from bs_batch_offsets).  The scatter map is the
 * concatenation of each instance's map, with ids relative to that
 * instance's own global nodes. */

/* Box mesh of E elements at degree N: the first E elements of the m^3
 * element box (m the smallest with m^3 >= E) in lexicographic order,
 * identity orientation; local numbering as bs_mesh_hex_map; the global
 * nodes are the lattice points the elements touch, numbered by rank in
 * lattice order (X fastest).  map: host int32[E (N+1)^3]; *n_global gets
 * the node count.  Host only. */
bs_status bs_mesh_box_map_host(int64_t E, int N, int32_t* map, int64_t* n_global);

typedef struct bs_batch bs_batch;

/* Build a batch of n_inst instances from host arrays h_n_local[n_inst],
 * h_n_global[n_inst] and the concatenated device map d_map (int32, sum of
 * n_local entries).  Totals must stay below 2^31.  Allocates, synchronises
 * `stream`; BS_ERR_INVALID_ARG if a map id lies outside its instance. */
bs_status bs_batch_create(bs_ctx* ctx, int32_t n_inst, const int64_t* h_n_local, const int64_t* h_n_global,
                          const int32_t* d_map, void* stream, bs_batch** out);
bs_status bs_batch_destroy(bs_batch* batch);

/* Totals, chunk counts (chunks of 2048 entries never cross an instance) and
 * the workgroups of one persistent binary64 launch.  Any output pointer may
 * be NULL. */
bs_status bs_batch_info(const bs_batch* batch, int64_t* n_local, int64_t* n_global, int64_t* n_chunks_local,
                        int64_t* n_chunks_global, int32_t* persistent_blocks_f64);

/* Host int64[n_inst + 1] prefix offsets of the local and global vectors. */
bs_status bs_batch_offsets(const bs_batch* batch, int64_t* h_off_local, int64_t* h_off_global);

/* Nonzero if a wait of the persistent form ever outlived its limit (half a
 * second); the form then stops early and its results are invalid, and
 * later persistent steps on this batch do nothing.  Synchronises `stream`. */
bs_status bs_batch_barrier_timeouts(const bs_batch* batch, int32_t* count, void* stream);

/* Concatenated vectors of one batch step (all of the step's dtype): global
 * x, y, p, r, Ap (written, except that nothing writes x before reading it
 * in the same phase), local xL, pL (written) and wL (read). */
typedef struct {
  void* x;
  void* y;
  void* p;
  void* r;
  void* Ap;
  void* xL;
  void* pL;
  const void* wL;
} bs_batch_vectors;

enum {
  BS_BATCH_PER_INSTANCE = 0, /* eleven launches per instance               */
  BS_BATCH_PER_PHASE = 1,    /* eleven launches for the whole batch        */
  BS_BATCH_PERSISTENT = 2    /* one launch, work claimed in dependency order */
};

/* One step on every instance: the seven operations of Table 1 once each,
 * then one CG iteration (Algorithm 1) with A = Z^T Z:
 *   y = x;  y = alpha x + beta y;  norm = sum wL xL^2;  dot = x.y;
 *   x += alpha p, r -= alpha Ap, rr = r.r;  xL = Z x;  y = Z^T xL;
 *   pL = Z p;  Ap = Z^T pL;  pAp = p.Ap, a = rr/pAp;
 *   x += a p, r -= a Ap, rr2 = r.r;  p = r + (rr2/rr) p.
 * d_out: device binary64[n_inst * 8]; instance i gets norm, dot, rr, pAp, a,
 * rr2, rr2/rr in slots 0..6 (slot 7 untouched).  Reductions are compensated
 * per chunk and summed per instance in chunk order; the modes run the same
 * code on the same chunks and give identical bits.  Per-phase and
 * persistent steps neither allocate nor synchronise (graph-capturable).
 * Calls on one batch must not overlap (they share its partial sums and the
 * persistent form's schedule). */
bs_status bs_batch_step(bs_ctx* ctx, bs_batch* batch, bs_dtype dtype, int mode, const bs_batch_vectors* v,
                        double alpha, double beta, double* d_out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* BS_H */
