// Internal definitions of the gfx950 global-local multigrid library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <type_traits>
#include <string>
#include <utility>
#include <vector>

#include "mgpcg.h"

namespace mg {

// ---------------------------------------------------------------------------
// errors: internal code throws Error; the C entry points catch it.
// ---------------------------------------------------------------------------
struct Error {
  mg_status code;
  std::string msg;
};

[[noreturn]] void fail(mg_status code, const char *fmt, ...);

#define MG_HIP(call)                                                              \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess)                                                         \
      ::mg::fail(MG_ERR_HIP, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                 __FILE__, __LINE__);                                             \
  } while (0)

#define MG_LAUNCH_CHECK() MG_HIP(hipGetLastError())

// ---------------------------------------------------------------------------
// device buffer owning its allocation
// ---------------------------------------------------------------------------
template <class T>
struct DBuf {
  T *p = nullptr;
  size_t n = 0;
  DBuf() = default;
  DBuf(const DBuf &) = delete;
  DBuf &operator=(const DBuf &) = delete;
  DBuf(DBuf &&o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
  DBuf &operator=(DBuf &&o) noexcept {
    if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
    return *this;
  }
  ~DBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  void alloc(size_t count) {
    release();
    if (count == 0) return;
    hipError_t e = hipMalloc(reinterpret_cast<void **>(&p), count * sizeof(T));
    if (e != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      fail(MG_ERR_OOM, "hipMalloc of %zu bytes failed: %s", count * sizeof(T), hipGetErrorString(e));
    }
    n = count;
  }
  size_t bytes() const { return n * sizeof(T); }
  operator T *() const { return p; }
};

template <class T>
void upload(DBuf<T> &d, const T *h, size_t n, hipStream_t s) {
  d.alloc(n);
  if (n) MG_HIP(hipMemcpyAsync(d.p, h, n * sizeof(T), hipMemcpyHostToDevice, s));
}
template <class T>
void download(std::vector<T> &h, const T *d, size_t n, hipStream_t s) {
  h.resize(n);
  if (n) MG_HIP(hipMemcpyAsync(h.data(), d, n * sizeof(T), hipMemcpyDeviceToHost, s));
  MG_HIP(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------------------
// sliced ELL (SELL-C) with C = 64: one wavefront lane per row; inside a slice
// the entries of column position j of the 64 rows are contiguous.  Rows keep
// the order of the matrix they are built from: the length sorting of
// SELL-C-sigma is applied to the unknowns beforehand (Level::perm), so that
// row p of the layout is unknown p of every vector.
// ---------------------------------------------------------------------------
constexpr int SELL_C = 64;

struct Sell {
  int64_t nrows = 0, ncols = 0, nslices = 0, stored = 0;
  int sigma = 1;
  // gathers in flight per lane in the products with this matrix (4 or 8):
  // short rows run faster with 4 and twice the resident wavefronts, long rows
  // with 8; the solve-order autotuner times both on the level operator
  int unroll = 8;
  // 1: the products skip each row's padding past the slice's shortest row
  // (row lengths rlen, per-slice minimum smin); 0: they use every stored
  // entry.  Same result bitwise; the autotuner keeps the faster.
  int mask = 0;
  // lanes per row (1, 2, 4 or 8): a slice holds 64 / rpl rows, lane l works
  // on entries t, t + rpl, ... (t = l mod rpl) of row l / rpl of its slice;
  // long rows of small levels get rpl times the wavefronts
  int rpl = 1;
  DBuf<int64_t> slice_ptr;  // [nslices + 1]
  DBuf<int32_t> perm;       // [nslices * 64] row at each position, -1 = padding
  DBuf<uint16_t> rlen;      // [nslices * 64] entries held at each position, 0 = padding
  DBuf<int32_t> smin;       // [nslices] shortest row of each slice
  DBuf<int32_t> col;        // [stored]
  DBuf<double> v64;         // [stored] (FP64 copy)
  DBuf<float> v32;          // [stored] (FP32 copy, mixed precision)
  // 16-bit columns.  Per slice cbase = (base0, base1):
  //   base0 >= 0: two windows of 32768, column c stored as c - base0 (below
  //               0x8000) or 0x8000 | (c - base1);
  //   base0 = -2: up to 8 windows of 8192 starting at ctab[16 s + w], stored as
  //               (w << 13) | (c - ctab[16 s + w]);
  //   base0 = -3: up to 16 windows of 4096, (w << 12) | (c - ctab[16 s + w]);
  //   base0 = -1: 32-bit columns.
  DBuf<uint16_t> col16;     // [stored]
  DBuf<int32_t> cbase;      // [2 * nslices]
  DBuf<int32_t> ctab;       // [16 * nslices]
  int64_t nnz = 0, nnz16 = 0;  // entries, entries in 16-bit slices
};

struct Csr {
  int64_t nrows = 0, ncols = 0, nnz = 0;
  DBuf<int64_t> rowptr;
  DBuf<int32_t> col;
  DBuf<double> val;
};

// Symmetric inverses of a set of systems (the patches of a level, or the
// coarsest matrix) as the lower triangle of 32 x 32 tiles: tile (I, J), J <= I,
// of system k at tile_off[k] + (I (I + 1) / 2 + J) * 1024, row-major inside the
// tile, zero beyond the system size.  The apply runs over row items (system,
// tile row I, chunk of at most PACK_CHUNK tiles), each writing the row
// products of its chunk into one 32-entry slot of py and the transposed
// products of its off-diagonal tiles into pz (per system, column J of tile row
// I at zoff[k] + 32 (J nb - J (J + 1) / 2) + 32 (I - J - 1)), then over gather
// items (system, tile row J) that add them up in a fixed order.
constexpr int PATCH_TILE = 32;
constexpr int PACK_CHUNK = 16;  // default tiles per row item (chosen per level by timing)
struct PackedInv {
  int64_t packed = 0, ysize = 0, zsize = 0;
  int chunk = PACK_CHUNK;                       // tiles per row item: 8, 16 or 32
  DBuf<int64_t> tile_off, zoff;                 // [systems]
  DBuf<int32_t> r_sys, r_row, r_chunk, r_slot;  // row items
  DBuf<int32_t> g_sys, g_row, g_slot;           // gather items (first slot of the row)
  std::vector<int> colour_r_first, colour_g_first;  // [ncolour + 1]
  DBuf<double> v64;
  DBuf<float> v32;
};
void build_packed_layout(hipStream_t s, const std::vector<int32_t> &kptr, const std::vector<int> &colour_first,
                         PackedInv &P, int chunk = PACK_CHUNK);

// Patches of one level in kernel order (sorted by colour, then canonical id).
struct Patches {
  int n = 0, ncolour = 0, maxn = 0;
  int n_factor32 = 0;         // patches factored on the FP32 matrix cores
  int n_inherited = 0;        // components inherited from the finer level
  int64_t total = 0;          // sum of patch sizes
  std::vector<int> colour_first;   // [ncolour + 1] kernel-order patch ranges
  std::vector<int32_t> h_ptr, h_dofs, h_colour;  // canonical order (export)
  std::vector<int32_t> h_kptr;     // [n + 1] kernel-order offsets (host copy)
  DBuf<int32_t> ptr;          // [n + 1] kernel order
  DBuf<int32_t> dofs;         // [total] solve-order positions of the patch DOFs
  DBuf<int32_t> dofs_canon;   // [total] canonical free ids (factorisation)
  DBuf<int64_t> inv_off;      // [n] offset of the full inverse (n_d^2 entries, setup only)
  DBuf<double> inv64;         // full inverses, row-major (setup only)
  // Solve phase: the patch inverses, packed
  PackedInv inv;
  // rows of A at the patch DOFs (kernel order), columns in solve order
  Sell rows;
  // with patch_refine: the FP64 values of `rows` with every column outside
  // the row's own patch zeroed (A^[d] in the layout of rows), for the
  // refinement residual of the patch solves
  DBuf<double> loc;
  // tile rows per patch of the one-workgroup local correction
  // (patch_correct_small: 4, 8 or 12, i.e. patches of up to 128, 256 or 384
  // DOFs), 0 = the three-launch path; chosen per level by timing
  int small_nb = 0;
  // per colour: 1 if no patch row couples to a DOF of another patch of the
  // colour, so that one launch per colour (patch_correct_small without a
  // residual) equals the residual of all patches followed by all corrections
  std::vector<uint8_t> colour_fused;
  // the rows of A that couple to a patch DOF (ascending solve order) and their
  // solve-order positions: after the local correction from u = 0, u vanishes
  // outside the patch DOFs, so b - A u equals b on every other row
  Sell nbr;
  DBuf<int32_t> nbr_pos;
};

// The coarsest solve by nested dissection (coarse_nd.hip): supernodes
// (leaves and separators, contiguous ranges of the dissection order) with the
// inverses of their diagonal blocks of L and the nonzero 32-row tile rows of L
// below them, all FP64.
struct CoarseNd {
  bool on = false;
  int nsup = 0, height = 0, leaf = 0;
  int64_t dinv_bytes = 0, b_bytes = 0;
  DBuf<int32_t> pos;                      // [n] dissection order -> unknown
  DBuf<int32_t> t_sup, t_loc;             // per global tile
  DBuf<int32_t> s_a, s_n, s_t0;           // per supernode
  DBuf<int64_t> s_doff;
  DBuf<double> dinv;                      // diagonal-block inverses, lower tiles
  DBuf<int32_t> q_sup, q_tgt;             // per stored tile row
  DBuf<int64_t> q_off;
  DBuf<double> bval;
  DBuf<int32_t> s_qptr, s_q, g_qptr, g_q;
  std::vector<int> lvl_tiles_first, lvl_items_first;  // by tree height
  DBuf<int32_t> lvl_tiles, lvl_items;
  DBuf<double> bp, y, t, x, contrib;      // solve work
};

struct Level {
  // mesh and DOF map
  int dim = 0, degree = 0, nloc = 0;
  int64_t nv = 0, nc = 0, ne = 0, ndofs = 0, nfree = 0;
  // unknowns per DOF node (dim for elasticity) and the number of free DOF
  // nodes; nfree = ncomp * nfree_s counts the unknowns of the level
  int ncomp = 1;
  int64_t nfree_s = 0;
  DBuf<double> coords;
  DBuf<int32_t> cells;
  DBuf<uint8_t> dirv;
  DBuf<int32_t> cell_dofs;     // [nc * nloc]
  DBuf<int32_t> free_index;    // [ndofs] -> free id or -1
  DBuf<int32_t> free_dofs;     // [nfree] -> canonical id
  DBuf<double> nodes;          // [ndofs * dim]
  DBuf<double> gamma;
  DBuf<uint8_t> flags;
  int64_t nflagged = 0;
  double gamma_min = 0;
  // operator: A in canonical free order (export, Galerkin product, patch
  // gathers); S is A in solve order: unknown p of every solve-phase vector is
  // canonical unknown perm[p], rows sorted by length inside sigma windows
  Csr A;
  Sell S;
  DBuf<int32_t> perm, iperm;   // solve order <-> canonical free order
  DBuf<double> dinv64;
  DBuf<float> dinv32;
  // transfer to the next coarser level (absent on the coarsest)
  int pw = 0;
  DBuf<int32_t> locate;        // [nfree]
  DBuf<int32_t> pcol;          // [nfree * pw] row-major, -1 = dropped
  DBuf<double> pval;           // [nfree * pw]
  Csr Pc, Rc;                  // P and R = P^T as CSR (Galerkin product)
  Sell P, R;                   // y += P x_c ; y = R r
  // local correction
  Patches patch;
  // multicolour symmetric Gauss-Seidel (global smoother option): the rows of
  // each colour as a SELL matrix (columns in solve order) and their solve-order
  // positions; the colour of every unknown in canonical order (export)
  std::vector<Sell> sgs;
  std::vector<DBuf<int32_t>> sgs_pos;
  DBuf<int32_t> sgs_colour;
  // Chebyshev
  double lam = 0, lam_adj = 0, lo = 0, hi = 0;
  int lanczos_steps = 0, lanczos_steps_adj = 0;
  // coarsest: dense inverse, or the nested-dissection factor
  bool coarsest = false;
  CoarseNd cnd;
  DBuf<double> cinv;           // [nfree * nfree] (setup only)
  PackedInv cpk;               // the coarsest inverse, packed (one system)
  DBuf<int32_t> cptr;          // {0, nfree}
  DBuf<double> cpy, cpz;       // its apply partial products
  // V-cycle work vectors, precision of the cycle
  DBuf<double> w64[6];
  DBuf<float> w32[6];
  DBuf<double> res64;          // patch residuals [patch.total]
  DBuf<float> res32;
  DBuf<double> py64, pz64;     // patch apply partial products [inv.ysize], [inv.zsize]
  DBuf<float> py32, pz32;
  DBuf<double> pst;            // patch_refine: staged first patch solves [nfree], zero between calls
  // the same for block solves: MG_BLOCK_MAX interleaved columns, allocated on
  // the first block solve
  DBuf<double> bw64[6];
  DBuf<float> bw32[6];
  DBuf<double> bres64;
  DBuf<float> bres32;
  double setup_ms = 0;
};

struct Ctx {
  mg_options opt{};
  double tau = 0.1;
  int layers = 1;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::vector<int32_t> layout;     // per-level fixed layout choices (4 per level)
  int device = 0;                  // device current at setup
  double *noalloc = nullptr;       // that device's static staging array (mg_vcycle_noalloc)
  std::vector<Level> lv;
  std::string err;
  // PCG work (FP64, level 0, solve order)
  DBuf<double> r, z, p, q, ax, bpos, xpos;
  DBuf<double> partial;        // dot-product block partials
  DBuf<double> scal;           // device scalars of CG (16 per column)
  double *h_scal = nullptr;    // pinned host mirror
  double *h_scal_dev = nullptr;  // its device address
  // mass matrix (free rows x all DOFs) for mg_rhs_from_nodal, built lazily
  Csr M;
  Sell Ms;
  // kernel timing
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
  std::vector<int> event_slot;          // level of each event pair
  size_t events_used = 0;
  std::vector<int64_t> timed_launches;  // per level
  std::vector<double> timed_ms;
  // captured V-cycle graph (mg_vcycle, mg_vcycle_solve)
  hipGraphExec_t graph_exec = nullptr;
  hipGraph_t graph = nullptr;
  // block CG work (FP64, level 0, solve order, MG_BLOCK_MAX interleaved
  // columns; allocated on the first block solve) and the captured CG
  // iterations (index: block width, 1 = the single-vector solve)
  DBuf<double> kr, kz, kp, kq, kx, kb, kpartial;
  hipGraphExec_t cg_exec[5] = {};
  hipGraph_t cg_graph[5] = {};
  ~Ctx();
};

// right-hand sides advanced together by one block solve
constexpr int MG_BLOCK_MAX = 4;

// ---------------------------------------------------------------------------
// setup stages (setup_*.hip)
// ---------------------------------------------------------------------------
void build_dofmap(Ctx &c, Level &L, const mg_mesh &m);
void compute_quality(Ctx &c, Level &L);
void assemble_fine(Ctx &c, Level &L);
void assemble_mass(Ctx &c, Level &L);
void build_prolongation(Ctx &c, Level &fine, const Level &coarse, const mg_mesh &cm);
void galerkin_product(Ctx &c, Level &fine, Level &coarse);
void build_patches(Ctx &c, Level &L, const mg_mesh &m);
void set_patches(Ctx &c, Level &L, const std::vector<std::vector<int32_t>> &dofs);
void patch_seeds(Ctx &c, Level &L, std::vector<std::vector<int32_t>> &seeds);
void inherit_patches(Ctx &c, const Level &F, Level &C, std::vector<std::vector<int32_t>> &seeds);
void factor_patches(Ctx &c, Level &L);
void factor_patches_batched(Ctx &c, Level &L, int batch_max, std::vector<int32_t> &rest, int *bad);
void build_patch_rows(Ctx &c, Level &L, bool want32);
void relayout_patch_rows(Ctx &c, Level &L, bool want32, int rpl);
void build_patch_refine(Ctx &c, Level &L);
void build_patch_neighbours(Ctx &c, Level &L, bool want32);
void build_sgs(Ctx &c, Level &L, bool want32);
void factor_coarsest(Ctx &c, Level &L);
void factor_coarsest_nd(Ctx &c, Level &L, int leaf);
template <class T>
void coarse_apply_nd(hipStream_t s, const Level &L, const T *b, T *u, int vs);
void estimate_eigenvalues(Ctx &c, Level &L);
void build_sell(Ctx &c, const Csr &A, Sell &S, int sigma, bool want32, int rpl = 1);
void ell_to_csr(Ctx &c, int64_t nrows, int64_t ncols, int width, const int32_t *col, const double *val,
                bool transpose, Csr &A);
void spgemm(Ctx &c, const Csr &A, const Csr &B, Csr &C);
// removes off-diagonal entries with |a_ij| <= 1e-12 sqrt(|a_ii a_jj|) (square A)
void drop_cancelled(Ctx &c, Csr &A);
void solve_order(Ctx &c, Level &L, int sigma, bool want32);
void build_transfer_sell(Ctx &c, Level &F, const Level &C, bool want32);
void permute_patches(Ctx &c, Level &L);
void ensure_work(Ctx &c, Level &L);

// ---------------------------------------------------------------------------
// solve-phase kernels (solve.hip)
// ---------------------------------------------------------------------------
template <class T>
void sell_spmv(hipStream_t s, const Sell &S, const T *x, T *y, int mode, const T *b);
// modes of sell_spmv
enum { SPMV_SET = 0, SPMV_ADD = 1, SPMV_RESID = 2 };

template <class T>
void cheb_step(hipStream_t s, const Sell &S, const T *dinv, const T *b, const T *x, T *xout, T *d,
               int first, double c_d, double c_r);
// The first Chebyshev step (d = c_r D^-1 (b - A x), x' = x + d; d not stored
// when d is NULL) from an x that vanishes outside the rows coupled by nbr:
// one pass over the vectors with A x = 0, then the full step on the nbr rows.
// nbr NULL: x = 0 everywhere (x is not read and may be NULL).
template <class T>
void cheb_step_zero(hipStream_t s, int64_t n, const Sell *nbr, const int32_t *nbr_pos, const T *dinv,
                    const T *b, const T *x, T *xout, T *d, double c_r);

template <class T>
void patch_residual(hipStream_t s, const Patches &pt, int colour, const T *b, const T *u, T *res);
// res, b and u are read and written at stride vs (one column of a block vector
// when vs > 1)
template <class T>
void patch_apply(hipStream_t s, const Patches &pt, int colour, const T *res, T *py, T *pz, T *u, int vs = 1);
// the same with one step of iterative refinement (FP64 residual of the patch
// systems); res is overwritten, st (n_free doubles, zero outside a call) stages
// the first solve
template <class T>
void patch_apply_refined(hipStream_t s, const Patches &pt, int colour, T *res, T *py, T *pz, T *u, double *st,
                         int vs = 1);
// Patches of at most SMALL_PATCH DOFs, one workgroup per patch, bitwise
// equal to patch_residual followed by patch_apply: with res = NULL the whole
// local correction of one colour (residual, product with the packed inverse,
// update of u) in one launch (colour_fused colours only); else the product
// and the update, from the residual res of patch_residual.
constexpr int SMALL_PATCH = 384;  // largest patch of the one-workgroup path (12 tile rows)
constexpr int MAX_PATCH = 16384;  // largest local-correction patch (its dense inverse: 2 GiB in FP64)
template <class T>
void patch_correct_small(hipStream_t s, const Patches &pt, int colour, const T *b, const T *res, T *u);
template <class T>
void coarse_apply(hipStream_t s, const Level &L, const T *b, T *u, int vs = 1);
template <class T>
void sgs_colour_sweep(hipStream_t s, const Sell &S, const int32_t *pos, const T *dinv, const T *b, T *u);


template <class T>
void fill(hipStream_t s, T *x, int64_t n, T v);
template <class A, class B>
void convert(hipStream_t s, const A *x, B *y, int64_t n);
void copy64(hipStream_t s, const double *x, double *y, int64_t n);
// y[p] = x[perm[p]] (to solve order) and y[perm[p]] = x[p] (back)
template <class A, class B>
void gather_perm(hipStream_t s, const A *x, const int32_t *perm, B *y, int64_t n);
template <class A, class B>
void scatter_perm(hipStream_t s, const A *x, const int32_t *perm, B *y, int64_t n);
void add64(hipStream_t s, double *y, const double *x, int64_t n);
int spmv_dot_blocks(const Sell &S);
void spmv_dot(hipStream_t s, const Sell &S, const double *p, double *q, double *part);

// dot products: partial sums into part, then finalisation into out[0]
void dot_partials(hipStream_t s, const double *x, const double *y, int64_t n, double *part,
                  int nblocks);
int dot_blocks(int64_t n);
void finish_sum(hipStream_t s, const double *part, int nblocks, double *out);

// ---------------------------------------------------------------------------
// block solve kernels (solve_block.hip): K in {2, 4} columns interleaved,
// unknown i of column q at index i K + q
// ---------------------------------------------------------------------------
template <class T>
void sell_spmv_block(hipStream_t s, const Sell &S, int K, const T *x, T *y, int mode, const T *b);
template <class T>
void cheb_step_block(hipStream_t s, const Sell &S, int K, const T *dinv, const T *b, const T *x, T *xout, T *d,
                     int flags, double c_d, double c_r);
template <class T>
void sgs_colour_sweep_block(hipStream_t s, const Sell &S, int K, const int32_t *pos, const T *dinv, const T *b,
                            T *u);
template <class T>
void patch_residual_block(hipStream_t s, const Patches &pt, int colour, int K, const T *b, const T *u, T *res);
template <class T>
void cheb_step_zero_block(hipStream_t s, int64_t n, int K, const Sell *nbr, const int32_t *nbr_pos, const T *dinv,
                          const T *b, const T *x, T *xout, T *d, double c_r);
void spmv_dot_block(hipStream_t s, const Sell &S, int K, const double *p, double *q, double *part);
void dot_partials_block(hipStream_t s, int K, const double *x, const double *y, int64_t n, double *part,
                        int nblocks);
void finish_sum_block(hipStream_t s, int K, const double *part, int nblocks, double *out);
void cg_alpha_block(hipStream_t s, int K, double *scal);
void cg_update_xr_block(hipStream_t s, int K, double *x, double *r, const double *p, const double *q,
                        const double *scal, int64_t n, double *part, int nblocks);
void cg_beta_block(hipStream_t s, int K, double *scal);
void cg_active_block(hipStream_t s, int K, unsigned mask, double *scal);
void cg_update_p_block(hipStream_t s, int K, double *p, const double *z, const double *scal, int64_t n);
// cols: host array of K device pointers (canonical order; NULL = zero column)
void gather_block(hipStream_t s, int K, const double *const *cols, const int32_t *perm, double *y, int64_t n);
void scatter_block(hipStream_t s, int K, const double *y, const int32_t *perm, double *const *cols, int64_t n);

// CG helpers working on device scalars
void cg_alpha(hipStream_t s, double *scal);
void cg_update_xr(hipStream_t s, double *x, double *r, const double *p, const double *q,
                  const double *scal, int64_t n, double *part, int nblocks);
void cg_beta(hipStream_t s, double *scal);
void cg_update_p(hipStream_t s, double *p, const double *z, const double *scal, int64_t n);
void scal_to_host(hipStream_t s, const double *scal, double *host_dev, int count);

}  // namespace mg
