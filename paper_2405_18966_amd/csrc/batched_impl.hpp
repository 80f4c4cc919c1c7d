// Batched solver: many independent CSR problems with the same options run
// Alg. 2 in lockstep, each launch serving every problem (included by
// solver.hip, which provides the plan machinery).
//
// The problems are stacked as one block-diagonal matrix (segments padded to
// 256 rows, see kernels_batch.hpp).  A plan of that matrix supplies the
// device CSC copy, the product work items (tagged with their problem), the
// bases and the vectors; products therefore run unchanged, with per-problem
// scale factors.  Everything that reduces over a vector (CGS2 projections,
// norms, residuals) is segmented per problem; the small SVDs run one
// workgroup per problem.  A problem whose test passes is frozen at the next
// restart: the restart rotation puts its Ritz vectors in the leading basis
// columns, its restart panels become the identity (later rotations copy those
// columns exactly) and every kernel skips its work from then on; the outputs
// are formed for all problems at the end.
namespace svds {

struct BSrc {
  const int32_t *rp, *ci;
  const void *val;
  int64_t m, nnz, mo, nzo, no, mp;
};

// Stacked CSR: rows of problem b at [mo, mo + mp) (padding rows empty),
// columns shifted by no, values copied.  Grid (x, problems).
template <typename TV>
static __global__ void stack_csr_kernel(const BSrc *__restrict__ src, int32_t *__restrict__ rp,
                                        int32_t *__restrict__ ci, TV *__restrict__ val) {
  const BSrc s = src[blockIdx.y];
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  const int64_t t0 = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  for (int64_t i = t0; i < s.mp; i += stride)
    rp[s.mo + i] = static_cast<int32_t>(s.nzo + (i <= s.m ? s.rp[i] : s.nnz));
  for (int64_t z = t0; z < s.nnz; z += stride) {
    ci[s.nzo + z] = static_cast<int32_t>(s.ci[z] + s.no);
    val[s.nzo + z] = static_cast<const TV *>(s.val)[z];
  }
}

static __global__ void set_last_rowptr_kernel(int32_t *rp, int64_t row, int32_t v) { rp[row] = v; }

// S_b[c] = sig[b k + c]
static __global__ void bcopy_sig_kernel(int k, const double *__restrict__ sig, double *const *__restrict__ S) {
  const int b = blockIdx.x;
  for (int c = threadIdx.x; c < k; c += blockDim.x) S[b][c] = sig[static_cast<int64_t>(b) * k + c];
}

struct Batch {
  svds_plan *P = nullptr;
  int nb = 0;
  std::vector<BProb> hp;
  int64_t Mtot = 0, Ntot = 0, MT = 0, NT = 0;
  char *mem = nullptr;  // one device allocation for everything below
  BProb *dp = nullptr;
  int32_t *tile_u = nullptr, *tile_v = nullptr;
  int32_t *rp = nullptr, *ci = nullptr;
  void *val = nullptr;
  int64_t *v0o = nullptr;
  double *T = nullptr, *xs_u = nullptr, *xs_v = nullptr, *ones = nullptr, *coef = nullptr, *sigma_est = nullptr;
  double *rho = nullptr, *sig = nullptr, *res = nullptr, *Uk = nullptr, *Vext = nullptr, *yt = nullptr;
  double *npart = nullptr, *resid_av = nullptr, *resid_atu = nullptr, *Uc = nullptr, *Vc = nullptr;
  double *tmp_m = nullptr, *tmp_n = nullptr, *ones_k = nullptr;
  double *h1 = nullptr, *h2 = nullptr, *part = nullptr, *rho_b = nullptr;  // basis-typed scratch (<= 8 B)
  int *flags = nullptr, *bd = nullptr;
  int32_t *active = nullptr, *freeze = nullptr;  // per-problem work mask, problems to freeze
  double **optr = nullptr;  // output pointer tables U[nb], V[nb], S[nb]
  int *h_flags = nullptr;   // pinned, 4 per problem
  // work lists of the active problems (rebuilt when the active set changes):
  // product items of A and A^T, U-side and V-side tiles
  char *wl_mem = nullptr;
  int4 *wl_items[2] = {};
  int32_t *wl_tiles[2] = {};
  int wl_ntiles[2] = {};
  std::vector<int> item_prob[2];  // problem of each full-list item
  std::vector<int4> h_wl_items;
  std::vector<int32_t> h_wl_tiles;
  std::vector<int32_t> h_active;
  std::vector<int> conv_cycle;  // cycle (of the current phase) at which each problem converged
  uint64_t wl_version = 0;      // bumped whenever the work lists change (captured cycles key on it)
  ~Batch() {
    if (P) svds_plan_destroy(P);
    if (mem) (void)hipFree(mem);
    if (wl_mem) (void)hipFree(wl_mem);
    if (h_flags) (void)hipHostFree(h_flags);
  }
};

#define B_LAUNCH_CHECK() HIP_TRY(hipGetLastError())

template <typename TB, typename TO>
static int b_rotate(Batch &Bt, int side_v, int pc, int kc, const TB *Bm, int64_t ldb, const double *Y, int64_t ys,
                    int64_t ldy, TO *out, int64_t ldo) {
  svds_plan *P = Bt.P;
  const int ldyt = rot_ldyt(kc);
  const int64_t yts = static_cast<int64_t>(pc) * ldyt;
  ACC_BEFORE(SVDS_KC_ROTATE);
  hipLaunchKernelGGL(brot_transpose_kernel, dim3(static_cast<unsigned>(std::min<int64_t>(4096, ceil_div(yts * Bt.nb, 256)))),
                     dim3(256), 0, P->stream, Bt.nb, pc, kc, Y, ys, ldy, Bt.yt, yts, ldyt);
  const int32_t *tile = side_v ? Bt.tile_v : Bt.tile_u;
  const dim3 g(static_cast<unsigned>(side_v ? Bt.NT : Bt.MT));
#define BROT(K)                                                                                              \
  hipLaunchKernelGGL((brotate_kernel<TB, TO, K>), g, dim3(BT), 0, P->stream, pc, kc, Bm, ldb, Bt.yt, yts, ldyt, \
                     tile, out, ldo)
  if (kc <= 8) BROT(8);
  else if (kc <= 16) BROT(16);
  else if (kc <= 32) BROT(32);
  else BROT(64);
#undef BROT
  B_LAUNCH_CHECK();
  const double L = static_cast<double>(side_v ? Bt.Ntot : Bt.Mtot);
  ACC_AFTER(SVDS_KC_ROTATE, sizeof(TB) * L * (pc + kc), 2.0 * L * pc * kc);
  return SVDS_OK;
}

// CGS2 of w against Q[:, 0:j] per problem, norm, T entry (t_off, or -1),
// reciprocal scale xs (cf. cgs2_finish).
template <typename TB>
static int b_cgs2(Batch &Bt, Lanczos<TB> &Lz, int side_v, const TB *Q, int j, const TB *w, TB *w1, TB *out,
                  int mode, int64_t t_off, double *xs) {
  svds_plan *P = Bt.P;
  const int64_t L = side_v ? Bt.Ntot : Bt.Mtot, nt = side_v ? Bt.NT : Bt.MT;
  const int64_t ldq = side_v ? Lz.ldv : Lz.ldu;
  const int32_t *tile = side_v ? Bt.tile_v : Bt.tile_u;
  const int32_t *tl = Bt.wl_tiles[side_v];
  const unsigned ntl = static_cast<unsigned>(Bt.wl_ntiles[side_v]);
  TB *part = reinterpret_cast<TB *>(Bt.part);
  TB *h1 = reinterpret_cast<TB *>(Bt.h1), *h2 = reinterpret_cast<TB *>(Bt.h2);
  const double sb = sizeof(TB);
  const TB *src = w;
  if (j > 0) {
    ACC_BEFORE(SVDS_KC_CGS_PROJ);
    hipLaunchKernelGGL((bproj_kernel<TB>), dim3(ntl), dim3(BT), 0, P->stream, Q, ldq, j, w, tile, Bt.active, tl, nt,
                       part);
    B_LAUNCH_CHECK();
    ACC_AFTER(SVDS_KC_CGS_PROJ, sb * L * (j + 1), 2.0 * L * j);
    ACC_BEFORE(SVDS_KC_CGS_REDUCE);
    hipLaunchKernelGGL((bseg_sum_kernel<TB>), dim3(Bt.nb), dim3(BHJ), 0, P->stream, part, nt, j, Bt.dp, side_v,
                       Bt.active, h1, BHJ);
    B_LAUNCH_CHECK();
    ACC_AFTER(SVDS_KC_CGS_REDUCE, sb * nt * j, 0.0);
    ACC_BEFORE(SVDS_KC_CGS_UPDPROJ);
    if (j <= 32)
      hipLaunchKernelGGL((bupd_proj_kernel<TB, 32>), dim3(ntl), dim3(BT), 0, P->stream, Q, ldq, j, w, h1, BHJ, tile,
                         Bt.active, tl, nt, w1, part);
    else
      hipLaunchKernelGGL((bupd_proj_kernel<TB, 64>), dim3(ntl), dim3(BT), 0, P->stream, Q, ldq, j, w, h1, BHJ, tile,
                         Bt.active, tl, nt, w1, part);
    B_LAUNCH_CHECK();
    ACC_AFTER(SVDS_KC_CGS_UPDPROJ, sb * L * (j + 2), 4.0 * L * j);
    ACC_BEFORE(SVDS_KC_CGS_REDUCE);
    hipLaunchKernelGGL((bseg_sum_kernel<TB>), dim3(Bt.nb), dim3(BHJ), 0, P->stream, part, nt, j, Bt.dp, side_v,
                       Bt.active, h2, BHJ);
    B_LAUNCH_CHECK();
    ACC_AFTER(SVDS_KC_CGS_REDUCE, sb * nt * j, 0.0);
    src = w1;
  }
  ACC_BEFORE(SVDS_KC_CGS_UPDNORM);
  hipLaunchKernelGGL((bupd_norm_kernel<TB>), dim3(ntl), dim3(BT), 0, P->stream, Q, ldq, j, src, h2, BHJ, tile,
                     Bt.active, tl, out, Bt.npart);
  B_LAUNCH_CHECK();
  ACC_AFTER(SVDS_KC_CGS_UPDNORM, sb * L * (j + 2), 2.0 * L * j + 2.0 * L);
  ACC_BEFORE(SVDS_KC_CGS_REDUCE);
  hipLaunchKernelGGL((bfinish_norm_kernel<TB>), dim3(Bt.nb), dim3(CGS_THREADS), 0, P->stream, Bt.npart, Bt.dp,
                     side_v, Bt.active, mode, t_off >= 0 ? Bt.T + t_off * Bt.nb : nullptr, xs, Bt.sigma_est, Bt.bd,
                     P->opts.seed, Q, ldq, j, out);
  B_LAUNCH_CHECK();
  ACC_AFTER(SVDS_KC_CGS_REDUCE, 8.0 * nt, 0.0);
  return SVDS_OK;
}

template <typename TB> static int b_lanczos(Batch &Bt, Lanczos<TB> &Lz, int i0) {
  svds_plan *P = Bt.P;
  const int p = P->p, ld = p + 1;
  const int64_t nb = Bt.nb;
  TB *U = Lz.U[Lz.cur], *V = Lz.V[Lz.cur];
  for (int i = i0; i < p; ++i) {
    int rc = matvec<TB>(P, true, Lz.bu, Bt.xs_u, Bt.T + (i * ld + i) * nb, V + i * Lz.ldv, Lz.wv, U + i * Lz.ldu,
                        Bt.Mtot);
    if (rc) return rc;
    rc = b_cgs2<TB>(Bt, Lz, 1, V, i + 1, Lz.wv, Lz.w1v, Lz.bv, MODE_LANCZOS, i * ld + i + 1, Bt.xs_v);
    if (rc) return rc;
    if (i == p - 1) {
      hipLaunchKernelGGL((bscale_copy_kernel<TB>), dim3(static_cast<unsigned>(std::min<int64_t>(4096, Bt.NT))),
                         dim3(BT), 0, P->stream, Bt.Ntot, Bt.tile_v, Bt.active, Lz.bv, Bt.xs_v, V + p * Lz.ldv);
      B_LAUNCH_CHECK();
      break;
    }
    rc = matvec<TB>(P, false, Lz.bv, Bt.xs_v, Bt.T + (i * ld + i + 1) * nb, U + i * Lz.ldu, Lz.wu,
                    V + (i + 1) * Lz.ldv, Bt.Ntot);
    if (rc) return rc;
    rc = b_cgs2<TB>(Bt, Lz, 0, U, i + 1, Lz.wu, Lz.w1u, Lz.bu, MODE_LANCZOS, (i + 1) * ld + i + 1, Bt.xs_u);
    if (rc) return rc;
  }
  return SVDS_OK;
}

// v0: caller's unpadded concatenation (v0_padded false), a padded stacked
// FP64 vector (true), or null (Philox per problem).
template <typename TB> static int b_start(Batch &Bt, Lanczos<TB> &Lz, const double *v0, bool v0_padded) {
  svds_plan *P = Bt.P;
  Lz.cur = 0;
  if (v0 && v0_padded)
    hipLaunchKernelGGL((cast_copy_kernel<double, TB>), dim3(ceil_div(Bt.Ntot, 256)), dim3(256), 0, P->stream,
                       Bt.Ntot, v0, Lz.w1v);
  else
    hipLaunchKernelGGL((bstart_kernel<TB>), dim3(static_cast<unsigned>(std::min<int64_t>(4096, Bt.NT))), dim3(BT), 0,
                       P->stream, Bt.Ntot, Bt.tile_v, Bt.dp, P->opts.seed, v0, Bt.v0o, Lz.w1v);
  B_LAUNCH_CHECK();
  int rc = b_cgs2<TB>(Bt, Lz, 1, nullptr, 0, Lz.w1v, nullptr, Lz.bv, MODE_NORM, -1, Bt.xs_v);
  if (rc) return rc;
  rc = matvec<TB>(P, false, Lz.bv, Bt.xs_v, nullptr, nullptr, Lz.wu, Lz.V[0], Bt.Ntot);
  if (rc) return rc;
  return b_cgs2<TB>(Bt, Lz, 0, nullptr, 0, Lz.wu, nullptr, Lz.bu, MODE_LANCZOS, 0, Bt.xs_u);
}

// Small SVDs of every problem; h_flags[4b] = converged, [4b+1] = leading count.
static int b_small_svd(Batch &Bt, double tol, bool &all_conv) {
  svds_plan *P = Bt.P;
  const int p = P->p, k = P->k;
  ACC_BEFORE(SVDS_KC_SMALLSVD);
  hipLaunchKernelGGL(bsmall_svd_kernel, dim3(Bt.nb), dim3(small_svd_threads(p)),
                     small_svd_lds_bytes(p), P->stream, Bt.T, Bt.nb, p, k, tol, Bt.Uk, Bt.Vext, Bt.sig, Bt.res,
                     Bt.rho, Bt.flags, Bt.sigma_est, Bt.active);
  B_LAUNCH_CHECK();
  ACC_AFTER(SVDS_KC_SMALLSVD, 16.0 * (p + 1) * (p + 1) * Bt.nb, 0.0);
  HIP_TRY(hipMemcpyAsync(Bt.h_flags, Bt.flags, sizeof(int) * 4 * Bt.nb, hipMemcpyDeviceToHost, P->stream));
  HIP_TRY(hipStreamSynchronize(P->stream));
  all_conv = true;
  for (int b = 0; b < Bt.nb; ++b) all_conv = all_conv && Bt.h_flags[4 * b] != 0;
  return P->acc.harvest();
}

// Work lists of the active problems: the product items of A and A^T (items
// are grouped by problem) and the U-side / V-side tiles; an empty list gets
// one inert entry (an empty item; a tile of an inactive problem).  Uploaded
// synchronously (the host staging vectors are reused).
static int b_update_worklists(Batch &Bt) {
  svds_plan *P = Bt.P;
  for (int t = 0; t < 2; ++t) {
    SpmvPlan &sp = t ? P->op.bwd : P->op.fwd;
    Bt.h_wl_items.clear();
    for (size_t i = 0; i < sp.h_items.size(); ++i)
      if (Bt.h_active[Bt.item_prob[t][i]]) Bt.h_wl_items.push_back(sp.h_items[i]);
    if (Bt.h_wl_items.empty()) Bt.h_wl_items.push_back(make_int4(0, 0, 0, 0));
    HIP_TRY(hipMemcpyAsync(Bt.wl_items[t], Bt.h_wl_items.data(), sizeof(int4) * Bt.h_wl_items.size(),
                           hipMemcpyHostToDevice, P->stream));
    sp.items = Bt.wl_items[t];
    sp.nitems = static_cast<int>(Bt.h_wl_items.size());
    HIP_TRY(hipStreamSynchronize(P->stream));
  }
  for (int side = 0; side < 2; ++side) {
    Bt.h_wl_tiles.clear();
    for (int b = 0; b < Bt.nb; ++b) {
      if (!Bt.h_active[b]) continue;
      const BProb &q = Bt.hp[b];
      const int32_t t0 = side ? q.tv0 : q.tu0, nt = side ? q.ntv : q.ntu;
      for (int32_t t = 0; t < nt; ++t) Bt.h_wl_tiles.push_back(t0 + t);
    }
    if (Bt.h_wl_tiles.empty()) Bt.h_wl_tiles.push_back(0);
    HIP_TRY(hipMemcpyAsync(Bt.wl_tiles[side], Bt.h_wl_tiles.data(), sizeof(int32_t) * Bt.h_wl_tiles.size(),
                           hipMemcpyHostToDevice, P->stream));
    Bt.wl_ntiles[side] = static_cast<int>(Bt.h_wl_tiles.size());
    HIP_TRY(hipStreamSynchronize(P->stream));
  }
  // side task of A v writes V-side rows, of A^T u U-side rows
  P->op.fwd.side_tiles = Bt.wl_tiles[1];
  P->op.fwd.side_ntiles = Bt.wl_ntiles[1];
  P->op.bwd.side_tiles = Bt.wl_tiles[0];
  P->op.bwd.side_ntiles = Bt.wl_ntiles[0];
  ++Bt.wl_version;
  return SVDS_OK;
}

// Problems whose test passed at the last small SVD and that are still
// active: their Ritz vectors are now in the leading basis columns (the
// restart rotation just ran); freeze them.
static int b_freeze_converged(Batch &Bt) {
  svds_plan *P = Bt.P;
  std::vector<int32_t> fz(Bt.nb, 0);
  bool any = false;
  for (int b = 0; b < Bt.nb; ++b)
    if (Bt.h_active[b] && Bt.h_flags[4 * b]) fz[b] = 1, Bt.h_active[b] = 0, any = true;
  if (!any) return SVDS_OK;
  HIP_TRY(hipMemcpyAsync(Bt.freeze, fz.data(), sizeof(int32_t) * Bt.nb, hipMemcpyHostToDevice, P->stream));
  hipLaunchKernelGGL(bfreeze_kernel, dim3(Bt.nb), dim3(256), 0, P->stream, Bt.nb, Bt.freeze, Bt.active, Bt.Uk, Bt.Vext,
                     P->p, P->k);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(P->stream));  // fz is a host temporary
  return b_update_worklists(Bt);
}

static int b_activate_all(Batch &Bt) {
  svds_plan *P = Bt.P;
  Bt.h_active.assign(Bt.nb, 1);
  HIP_TRY(hipMemcpyAsync(Bt.active, Bt.h_active.data(), sizeof(int32_t) * Bt.nb, hipMemcpyHostToDevice, P->stream));
  HIP_TRY(hipStreamSynchronize(P->stream));
  return b_update_worklists(Bt);
}

// Alg. 2 steps 8-9 for every active problem: Ritz vectors into the other
// ping-pong buffer (V[:, k] = v_{p+1}), then the converged problems freeze.
template <typename TB> static int b_restart_rotate(Batch &Bt, Lanczos<TB> &Lz) {
  svds_plan *P = Bt.P;
  const int p = P->p, k = P->k;
  const int nxt = 1 - Lz.cur;
  TB *U = Lz.U[Lz.cur], *V = Lz.V[Lz.cur];
  TB *Un = Lz.U[nxt], *Vn = Lz.V[nxt];
  int rc = b_rotate<TB, TB>(Bt, 0, p, k, U, Lz.ldu, Bt.Uk, static_cast<int64_t>(p) * k, p, Un, Lz.ldu);
  if (rc) return rc;
  rc = b_rotate<TB, TB>(Bt, 1, p + 1, k + 1, V, Lz.ldv, Bt.Vext, static_cast<int64_t>(p + 1) * (k + 1), p + 1, Vn,
                        Lz.ldv);
  if (rc) return rc;
  Lz.cur = nxt;
  return b_freeze_converged(Bt);
}

// Alg. 2 steps 10-11 (eq. (7)): u_{k+1} = A v_{k+1} - Uk rho, re-orthogonalized
// against Uk, alpha_{k+1}.  Only launches: this and the Lanczos steps after it
// form the captured part of a cycle.
template <typename TB> static int b_restart_tail(Batch &Bt, Lanczos<TB> &Lz) {
  svds_plan *P = Bt.P;
  const int p = P->p, k = P->k, ld = p + 1;
  TB *Un = Lz.U[Lz.cur], *Vn = Lz.V[Lz.cur];
  int rc = matvec<TB>(P, false, Vn + k * Lz.ldv, Bt.ones, nullptr, nullptr, Lz.wu, nullptr, 0);
  if (rc) return rc;
  TB *rho_b = reinterpret_cast<TB *>(Bt.rho_b);
  hipLaunchKernelGGL((cast_copy_kernel<double, TB>), dim3(ceil_div(static_cast<int64_t>(Bt.nb) * k, 256)), dim3(256),
                     0, P->stream, static_cast<int64_t>(Bt.nb) * k, Bt.rho, rho_b);
  ACC_BEFORE(SVDS_KC_OTHER);
  hipLaunchKernelGGL((bupd_norm_kernel<TB>), dim3(static_cast<unsigned>(Bt.wl_ntiles[0])), dim3(BT), 0, P->stream, Un,
                     Lz.ldu, k, Lz.wu, rho_b, k, Bt.tile_u, Bt.active, Bt.wl_tiles[0], Lz.w1u,
                     static_cast<double *>(nullptr));
  B_LAUNCH_CHECK();
  ACC_AFTER(SVDS_KC_OTHER, sizeof(TB) * double(Bt.Mtot) * (k + 2), 2.0 * Bt.Mtot * k);
  return b_cgs2<TB>(Bt, Lz, 0, Un, k, Lz.w1u, Lz.wu, Lz.bu, MODE_LANCZOS, static_cast<int64_t>(k) * ld + k, Bt.xs_u);
}

template <typename TB>
static int b_run_cycles(Batch &Bt, Lanczos<TB> &Lz, double tol_c, int maxit, bool stagnate, int &cycles,
                        bool &conv) {
  svds_plan *P = Bt.P;
  cycles = 0;
  conv = false;
  double best = INFINITY;
  int nodec = 0;
  const int k = P->k;
  Bt.conv_cycle.assign(Bt.nb, 0);
  int rc = b_activate_all(Bt);
  if (rc) return rc;
  rc = b_lanczos<TB>(Bt, Lz, 0);
  while (rc == SVDS_OK) {
    ++cycles;
    rc = b_small_svd(Bt, tol_c, conv);
    if (rc) break;
    for (int b = 0; b < Bt.nb; ++b)
      if (Bt.h_active[b]) Bt.conv_cycle[b] = cycles;
    if (conv || cycles >= maxit) break;
    if (stagnate) {
      std::vector<double> r(static_cast<size_t>(Bt.nb) * k);
      HIP_TRY(hipMemcpy(r.data(), Bt.res, sizeof(double) * r.size(), hipMemcpyDeviceToHost));
      double mx = 0;
      for (double v : r) mx = std::max(mx, v);
      if (mx < best) best = mx, nodec = 0;
      else if (++nodec >= 2) break;
    }
    rc = b_restart_rotate<TB>(Bt, Lz);
    if (rc) break;
    if (P->opts.flags & SVDS_FLAG_GRAPH) {
      rc = run_graphed<TB>(P, Lz, Bt.wl_version, [&] {
        const int r = b_restart_tail<TB>(Bt, Lz);
        return r ? r : b_lanczos<TB>(Bt, Lz, k);
      });
    } else {
      rc = b_restart_tail<TB>(Bt, Lz);
      if (rc) break;
      rc = b_lanczos<TB>(Bt, Lz, k);
    }
  }
  return rc;
}

}  // namespace svds

extern "C" int svds_csr_solve_batched(int32_t count, const svds_csr *As, const svds_opts *opts, double *const *U,
                                      double *const *S, double *const *V, svds_info *infos) {
  SVDS_ABI_TRY
  using namespace svds;
  if (count < 0 || (count > 0 && (!As || !opts || !U || !S || !V))) return SVDS_EINVAL;
  if (count == 0) return SVDS_OK;
  const auto t0 = std::chrono::steady_clock::now();
  const int k = opts->k;
  const int p = opts->p > 0 ? opts->p : std::max(15, 3 * k);
  const int32_t vt = As[0].dtype;
  if (vt != SVDS_F64 && vt != SVDS_F32) return SVDS_EUNSUPPORTED;
  if (opts->precision != SVDS_PREC_FP64 && opts->precision != SVDS_PREC_MIXED) return SVDS_EINVAL;
  if (opts->flags & (SVDS_FLAG_SMALLEST | SVDS_FLAG_SELECTIVE_REORTH | SVDS_FLAG_PARTIAL_REORTH | SVDS_FLAG_HARMONIC))
    return SVDS_EUNSUPPORTED;
  if (k < 1 || p <= k) return SVDS_EINVAL;
  if (p > JAC_SMALL_P || k + 1 > 64) return SVDS_EUNSUPPORTED;
  Batch Bt;
  Bt.nb = count;
  Bt.hp.resize(count);
  std::vector<BSrc> src(count);
  int64_t mo = 0, no = 0, nzo = 0;
  for (int b = 0; b < count; ++b) {
    const svds_csr &A = As[b];
    if (A.dtype != vt) return SVDS_EINVAL;
    if (A.m < 1 || A.n < 1 || A.nnz < 0 || !A.row_ptr || (A.nnz > 0 && (!A.col_idx || !A.val))) return SVDS_EINVAL;
    if (p > A.m || p + 1 > A.n) return SVDS_EINVAL;
    if (!U[b] || !S[b] || !V[b]) return SVDS_EINVAL;
    const int64_t mp = ceil_div(A.m, BT) * BT, np = ceil_div(A.n, BT) * BT;
    BProb &q = Bt.hp[b];
    q.mo = mo;
    q.no = no;
    q.m = static_cast<int32_t>(A.m);
    q.n = static_cast<int32_t>(A.n);
    q.tu0 = static_cast<int32_t>(mo / BT);
    q.ntu = static_cast<int32_t>(mp / BT);
    q.tv0 = static_cast<int32_t>(no / BT);
    q.ntv = static_cast<int32_t>(np / BT);
    src[b] = BSrc{A.row_ptr, A.col_idx, A.val, A.m, A.nnz, mo, nzo, no, mp};
    mo += mp;
    no += np;
    nzo += A.nnz;
  }
  if (mo >= (int64_t(1) << 31) || no >= (int64_t(1) << 31) || nzo >= (int64_t(1) << 31)) return SVDS_EUNSUPPORTED;
  Bt.Mtot = mo;
  Bt.Ntot = no;
  Bt.MT = mo / BT;
  Bt.NT = no / BT;
  hipStream_t st = static_cast<hipStream_t>(opts->stream);
  const size_t vsz = vt == SVDS_F64 ? 8 : 4;
  // one allocation for the stacked matrix, the problem tables and the per-problem state
  Arena a;
  a.counting = true;
  for (int pass = 0; pass < 2; ++pass) {
    Bt.dp = a.take<BProb>(count);
    Bt.tile_u = a.take<int32_t>(Bt.MT);
    Bt.tile_v = a.take<int32_t>(Bt.NT);
    Bt.rp = a.take<int32_t>(mo + 1);
    Bt.ci = a.take<int32_t>(std::max<int64_t>(1, nzo));
    Bt.val = a.take<char>(std::max<int64_t>(1, nzo) * vsz);
    Bt.v0o = a.take<int64_t>(count);
    const int64_t nb = count;
    Bt.T = a.take<double>(static_cast<size_t>((p + 1) * (p + 1) * nb));
    Bt.xs_u = a.take<double>(nb);
    Bt.xs_v = a.take<double>(nb);
    Bt.ones = a.take<double>(nb);
    Bt.coef = a.take<double>(nb);
    Bt.sigma_est = a.take<double>(nb);
    Bt.rho = a.take<double>(nb * k);
    Bt.rho_b = a.take<double>(nb * k);
    Bt.sig = a.take<double>(nb * k);
    Bt.res = a.take<double>(nb * k);
    Bt.Uk = a.take<double>(nb * p * k);
    Bt.Vext = a.take<double>(nb * (p + 1) * (k + 1));
    Bt.yt = a.take<double>(nb * rot_yt_doubles(p + 1, k + 1));
    Bt.npart = a.take<double>(std::max(Bt.MT, Bt.NT));
    Bt.resid_av = a.take<double>(nb * k);
    Bt.resid_atu = a.take<double>(nb * k);
    Bt.Uc = a.take<double>(mo * k);
    Bt.Vc = a.take<double>(no * k);
    Bt.tmp_m = a.take<double>(mo);
    Bt.tmp_n = a.take<double>(no);
    Bt.ones_k = a.take<double>(k);
    Bt.h1 = a.take<double>(nb * BHJ);
    Bt.h2 = a.take<double>(nb * BHJ);
    Bt.part = a.take<double>(static_cast<size_t>(BHJ) * std::max(Bt.MT, Bt.NT));
    Bt.flags = a.take<int>(4 * nb);
    Bt.bd = a.take<int>(nb);
    Bt.active = a.take<int32_t>(nb);
    Bt.freeze = a.take<int32_t>(nb);
    Bt.optr = a.take<double *>(3 * nb);
    if (pass == 0) {
      const size_t bytes = a.used;
      if (hipMalloc(&Bt.mem, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return SVDS_ENOMEM;
      }
      a = Arena{};
      a.base = Bt.mem;
      a.size = bytes;
      a.counting = false;
    }
  }
  // problem tables, tile maps, stacked CSR
  std::vector<int32_t> tu(Bt.MT), tv(Bt.NT);
  std::vector<int64_t> v0o(count);
  int64_t vo = 0;
  for (int b = 0; b < count; ++b) {
    for (int t = 0; t < Bt.hp[b].ntu; ++t) tu[Bt.hp[b].tu0 + t] = b;
    for (int t = 0; t < Bt.hp[b].ntv; ++t) tv[Bt.hp[b].tv0 + t] = b;
    v0o[b] = vo;
    vo += Bt.hp[b].n;
  }
  std::vector<double *> optr(3 * count);
  for (int b = 0; b < count; ++b) optr[b] = U[b], optr[count + b] = V[b], optr[2 * count + b] = S[b];
  BSrc *dsrc = nullptr;
  HIP_TRY(hipMalloc(&dsrc, sizeof(BSrc) * count));
  struct FreeSrc {
    BSrc *p;
    ~FreeSrc() { (void)hipFree(p); }
  } fs{dsrc};
  HIP_TRY(hipMemcpyAsync(dsrc, src.data(), sizeof(BSrc) * count, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(Bt.dp, Bt.hp.data(), sizeof(BProb) * count, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(Bt.tile_u, tu.data(), sizeof(int32_t) * Bt.MT, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(Bt.tile_v, tv.data(), sizeof(int32_t) * Bt.NT, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(Bt.v0o, v0o.data(), sizeof(int64_t) * count, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(Bt.optr, optr.data(), sizeof(double *) * 3 * count, hipMemcpyHostToDevice, st));
  {
    const dim3 g(64, count);
    if (vt == SVDS_F64)
      hipLaunchKernelGGL((stack_csr_kernel<double>), g, dim3(256), 0, st, dsrc, Bt.rp, Bt.ci,
                         static_cast<double *>(Bt.val));
    else
      hipLaunchKernelGGL((stack_csr_kernel<float>), g, dim3(256), 0, st, dsrc, Bt.rp, Bt.ci,
                         static_cast<float *>(Bt.val));
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(set_last_rowptr_kernel, dim3(1), dim3(1), 0, st, Bt.rp, mo, static_cast<int32_t>(nzo));
    HIP_TRY(hipGetLastError());
    std::vector<double> one(count, 1.0), onek(k, 1.0 / std::sqrt(static_cast<double>(k)));
    HIP_TRY(hipMemcpyAsync(Bt.ones, one.data(), sizeof(double) * count, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(Bt.ones_k, onek.data(), sizeof(double) * k, hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
  }
  // plan of the stacked matrix (device CSC, items per problem, bases)
  svds_csr big{mo, no, nzo, Bt.rp, Bt.ci, Bt.val, vt};
  svds_opts o = *opts;
  o.p = p;
  o.v0 = nullptr;
  std::vector<int64_t> seg_r(count), seg_c(count);
  for (int b = 0; b < count; ++b) {
    seg_r[b] = Bt.hp[b].mo + static_cast<int64_t>(Bt.hp[b].ntu) * BT;
    seg_c[b] = Bt.hp[b].no + static_cast<int64_t>(Bt.hp[b].ntv) * BT;
  }
  int rc = plan_create_csr_impl(&big, &o, &Bt.P, seg_r.data(), seg_c.data(), count);
  if (rc) return rc;
  svds_plan *P = Bt.P;
  P->op.fwd.x_tile_inst = Bt.tile_v;
  P->op.bwd.x_tile_inst = Bt.tile_u;
  P->op.fwd.active = Bt.active;
  P->op.bwd.active = Bt.active;
  {
    // problem of every product item, and the work-list buffers
    for (int t = 0; t < 2; ++t) {
      const SpmvPlan &sp = t ? P->op.bwd : P->op.fwd;
      Bt.item_prob[t].resize(sp.h_items.size());
      for (size_t i = 0; i < sp.h_items.size(); ++i) {
        const int4 it = sp.h_items[i];
        Bt.item_prob[t][i] = it.x >= 0 ? (it.w >> SPMV_CNT_BITS) : sp.h_long[-it.x - 1].inst;
      }
    }
    Arena wa;
    auto carve = [&](Arena &ar) {
      Bt.wl_items[0] = ar.take<int4>(std::max<size_t>(1, P->op.fwd.h_items.size()));
      Bt.wl_items[1] = ar.take<int4>(std::max<size_t>(1, P->op.bwd.h_items.size()));
      Bt.wl_tiles[0] = ar.take<int32_t>(std::max<int64_t>(1, Bt.MT));
      Bt.wl_tiles[1] = ar.take<int32_t>(std::max<int64_t>(1, Bt.NT));
    };
    carve(wa);
    if (hipMalloc(&Bt.wl_mem, wa.used) != hipSuccess) {
      (void)hipGetLastError();
      Bt.wl_mem = nullptr;
      return SVDS_ENOMEM;
    }
    wa = Arena{};
    wa.base = Bt.wl_mem;
    wa.counting = false;
    carve(wa);
  }
  HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&Bt.h_flags), sizeof(int) * 4 * count, hipHostMallocDefault));
  P->acc.reset();
  // ---- Alg. 2 for every problem ----
  HIP_TRY(hipMemsetAsync(Bt.sigma_est, 0, sizeof(double) * count, st));
  HIP_TRY(hipMemsetAsync(Bt.bd, 0, sizeof(int) * count, st));
  HIP_TRY(hipMemsetAsync(Bt.T, 0, sizeof(double) * (p + 1) * (p + 1) * count, st));
  bool conv = false;
  int cyc = 0;
  std::vector<int> cyc32(count, 0);
  if (P->mixed) {
    const double tol32 = std::max(P->tol, 1e-5);
    rc = b_activate_all(Bt);
    if (!rc) rc = b_start<float>(Bt, P->L32, opts->v0, false);
    if (!rc) rc = b_run_cycles<float>(Bt, P->L32, tol32, P->maxit, true, cyc, conv);
    P->cycles32 = cyc;
    cyc32 = Bt.conv_cycle;
    if (!rc) {
      // v1 of the FP64 phase: sum_j Vk(:, j) / sqrt(k) per problem, in FP64
      // (Vk = V32 Vh_k into Vc, then Vc times the constant k-vector)
      Lanczos<float> &L32 = P->L32;
      rc = b_rotate<float, double>(Bt, 1, p, k, L32.V[L32.cur], L32.ldv, Bt.Vext,
                                   static_cast<int64_t>(p + 1) * (k + 1), p + 1, Bt.Vc, Bt.Ntot);
      if (!rc) rc = b_rotate<double, double>(Bt, 1, k, 1, Bt.Vc, Bt.Ntot, Bt.ones_k, 0, k, Bt.tmp_n, Bt.Ntot);
    }
    if (!rc) {
      HIP_TRY(hipMemsetAsync(Bt.sigma_est, 0, sizeof(double) * count, st));
      HIP_TRY(hipMemsetAsync(Bt.T, 0, sizeof(double) * (p + 1) * (p + 1) * count, st));
      rc = b_activate_all(Bt);
      if (!rc) rc = b_start<double>(Bt, P->L64, Bt.tmp_n, true);
    }
    if (!rc) rc = b_run_cycles<double>(Bt, P->L64, P->tol, std::max(1, P->maxit - cyc), false, cyc, conv);
    P->cycles64 = cyc;
  } else {
    rc = b_activate_all(Bt);
    if (!rc) rc = b_start<double>(Bt, P->L64, opts->v0, false);
    if (!rc) rc = b_run_cycles<double>(Bt, P->L64, P->tol, P->maxit, false, cyc, conv);
    P->cycles64 = cyc;
  }
  if (rc) return rc;
  std::vector<int> cyc64 = Bt.conv_cycle;
  rc = b_activate_all(Bt);  // outputs and residuals for every problem
  if (rc) return rc;
  // ---- outputs (Alg. 2 steps 15-16), signs, FP64 residuals ----
  Lanczos<double> &Lz = P->L64;
  rc = b_rotate<double, double>(Bt, 1, p, k, Lz.V[Lz.cur], Lz.ldv, Bt.Vext, static_cast<int64_t>(p + 1) * (k + 1),
                                p + 1, Bt.Vc, Bt.Ntot);
  if (rc) return rc;
  if (!(opts->flags & SVDS_FLAG_NO_SIGNFIX)) {
    hipLaunchKernelGGL(bsign_kernel, dim3(k, count), dim3(256), 0, st, Bt.dp, Bt.Vc, Bt.Ntot, Bt.Uk, p, k);
    HIP_TRY(hipGetLastError());
  }
  rc = b_rotate<double, double>(Bt, 0, p, k, Lz.U[Lz.cur], Lz.ldu, Bt.Uk, static_cast<int64_t>(p) * k, p, Bt.Uc,
                                Bt.Mtot);
  if (rc) return rc;
  const bool resid = !(opts->flags & SVDS_FLAG_NO_RESIDUALS);
  if (resid) {
    for (int j = 0; j < k; ++j) {
      hipLaunchKernelGGL(bgather_kernel, dim3(ceil_div(count, 256)), dim3(256), 0, st, count, Bt.sig + j,
                         static_cast<int64_t>(k), Bt.coef);
      // A v_j - s_j u_j and A^T u_j - s_j v_j, norms per problem
      rc = matvec<double>(P, false, Bt.Vc + j * Bt.Ntot, Bt.ones, Bt.coef, Bt.Uc + j * Bt.Mtot, Bt.tmp_m, nullptr, 0,
                          SVDS_KC_OTHER);
      if (rc) return rc;
      hipLaunchKernelGGL((btile_sq_kernel<double>), dim3(Bt.MT), dim3(BT), 0, st, Bt.tmp_m, Bt.npart);
      hipLaunchKernelGGL(bseg_norm_kernel, dim3(count), dim3(CGS_THREADS), 0, st, Bt.npart, Bt.dp, 0,
                         Bt.resid_av + j, k);
      rc = matvec<double>(P, true, Bt.Uc + j * Bt.Mtot, Bt.ones, Bt.coef, Bt.Vc + j * Bt.Ntot, Bt.tmp_n, nullptr, 0,
                          SVDS_KC_OTHER);
      if (rc) return rc;
      hipLaunchKernelGGL((btile_sq_kernel<double>), dim3(Bt.NT), dim3(BT), 0, st, Bt.tmp_n, Bt.npart);
      hipLaunchKernelGGL(bseg_norm_kernel, dim3(count), dim3(CGS_THREADS), 0, st, Bt.npart, Bt.dp, 1,
                         Bt.resid_atu + j, k);
      HIP_TRY(hipGetLastError());
    }
  }
  hipLaunchKernelGGL(bcopy_out_kernel, dim3(64, count), dim3(256), 0, st, Bt.dp, 0, k, Bt.Uc, Bt.Mtot, Bt.optr);
  hipLaunchKernelGGL(bcopy_out_kernel, dim3(64, count), dim3(256), 0, st, Bt.dp, 1, k, Bt.Vc, Bt.Ntot,
                     Bt.optr + count);
  hipLaunchKernelGGL(bcopy_sig_kernel, dim3(count), dim3(64), 0, st, k, Bt.sig, Bt.optr + 2 * count);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(st));
  rc = P->acc.harvest();
  if (rc) return rc;
  const size_t nk = static_cast<size_t>(count) * k;
  std::vector<double> hs(nk), hres(nk), hav(nk, 0.0), hatu(nk, 0.0);
  std::vector<int> hbd(count);
  HIP_TRY(hipMemcpy(hs.data(), Bt.sig, sizeof(double) * nk, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(hres.data(), Bt.res, sizeof(double) * nk, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(hbd.data(), Bt.bd, sizeof(int) * count, hipMemcpyDeviceToHost));
  if (resid) {
    HIP_TRY(hipMemcpy(hav.data(), Bt.resid_av, sizeof(double) * nk, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(hatu.data(), Bt.resid_atu, sizeof(double) * nk, hipMemcpyDeviceToHost));
  }
  const double ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  int worst = SVDS_OK;
  for (int b = 0; b < count; ++b) {
    const bool cb = Bt.h_flags[4 * b] != 0;
    if (!cb) worst = SVDS_NOT_CONVERGED;
    if (!infos) continue;
    svds_info &in = infos[b];
    in = svds_info{};
    in.nconv = Bt.h_flags[4 * b + 1];
    in.cycles = cyc32[b] + cyc64[b];
    in.cycles_fp32 = cyc32[b];
    in.cycles_fp64 = cyc64[b];
    in.breakdowns = hbd[b];
    in.converged = cb ? 1 : 0;
    in.n_spmv = P->n_spmv;
    in.n_spmvT = P->n_spmvT;
    double me = 0, mt = 0, ma = 0;
    const double s1 = hs[static_cast<size_t>(b) * k];
    for (int j = 0; j < k; ++j) {
      const size_t i = static_cast<size_t>(b) * k + j;
      me = std::max(me, hres[i]);
      mt = std::max(mt, hatu[i] / std::max(hs[i], std::max(0x1.0p-52 * s1, 2.2250738585072014e-308)));
      ma = std::max(ma, hav[i] / std::max(s1, 2.2250738585072014e-308));
    }
    in.max_res_est = me;
    in.max_res_true = mt;
    in.max_res_av = ma;
    in.ms_total = ms;
    for (int c = 0; c < SVDS_KC_COUNT; ++c) {
      in.kc_ms[c] = P->acc.ms[c];
      in.kc_bytes[c] = P->acc.bytes[c];
      in.kc_flops[c] = P->acc.flops[c];
      in.kc_launches[c] = P->acc.launches[c];
      in.kc_sampled_launches[c] = P->acc.sampled[c];
      in.kc_sampled_bytes[c] = P->acc.sampled_bytes[c];
    }
    in.workspace_bytes = static_cast<int64_t>(P->arena.size + P->op.v32_bytes);
    in.graph_captures = static_cast<int32_t>(P->graphs.captures);
    in.graph_replays = static_cast<int32_t>(P->graphs.replays);
    in.tuning = P->tuning;
  }
  return worst;
  SVDS_ABI_CATCH
}
