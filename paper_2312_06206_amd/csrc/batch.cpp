// Batched S-ADI: many independent problems (their own N, alpha, kappa) advanced together.
// Instances are grouped by N; each group runs every phase of a step as one launch over all
// of its instances (blockIdx.y), and a run of steps can be replayed from a captured HIP
// graph.  Per group, the two line sweeps take the Gohberg-Semencul FFT kernels, two dense
// FP64 products with the explicit H^-1 (batched matrix-core products), or the same products
// in FP32 with one FP64 residual refinement; a timing pass picks the fastest.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <string>
#include <thread>
#include <vector>

#include "context.hpp"
#include "kernels.hpp"
#include "setup_math.hpp"

using namespace sadi_impl;

namespace {

struct Group {
  int n = 0, m = 0;
  std::vector<int> members;                   // instance indices
  sadi::BatchInst* d_inst = nullptr;          // device copy of the members' descriptors
  sadi::BatchInst* d_scratch_inst = nullptr;  // same, state in scratch buffers (timing)
  int path = SADI_PATH_FFT_GS;
  double ms[3] = {-1.0, -1.0, -1.0};          // timed ms per step for each path
  int tile[3] = {0, 0, 0};                    // tile of the dense products (0: by tile count)
  // dense path: H^-1 per member (rows H^-1 e_k) and the pointer triples of the two
  // products per member: T = X H^-1 into the spectrum buffer S (as real), then X = H^-1 T
  std::vector<double*> hinv;
  sadi::GemmPtrs* d_prod1 = nullptr;
  sadi::GemmPtrs* d_prod2 = nullptr;
  // FP32 dense path with one FP64 refinement (mixed_sweeps): H^-1 in FP32 and H in FP64 per
  // member; in the member's spectrum buffer: X32 and T32 (FP32, N x N each, later W in FP64)
  // and Y (FP64)
  sadi::GemmPtrs32<float>* d_m1 = nullptr;    // T32 = X32 Hinv32
  sadi::GemmPtrs32<double>* d_m2 = nullptr;   // Y = (or +=) H^-1 T32
  sadi::GemmPtrs* d_w = nullptr;              // W = Y H
  sadi::GemmPtrs* d_r = nullptr;              // X = X - H W
  sadi::CvtPtrs* d_cvt = nullptr;             // X32 = (float) X
  sadi::CopyPtrs* d_copy = nullptr;           // X = Y
  bool mixed_ready = false;                   // the above built (setup_mixed)
  bool dense_ready = false;                   // hinv, d_prod1, d_prod2 built (setup_dense)
};

bool dense_path(int path) { return path == SADI_PATH_DENSE || path == SADI_PATH_DENSE_MIXED; }

}  // namespace

struct sadi_batch {
  int magic = 0x5AD2;
  int count = 0;
  int dense_max_n = 0;                        // groups up to this N may take the dense paths
  hipStream_t stream = nullptr;
  hipStream_t own_stream = nullptr;
  std::vector<sadi_ctx*> ctx;
  std::vector<double*> u_prev, u_cur;
  std::vector<const double*> phi2;
  bool bound = false;
  std::vector<Group> groups;
  // descriptors of all instances (indexed like the creation arrays), bound state and the
  // tuner's scratch state, and the host copies they are uploaded from
  sadi::BatchInst* d_all = nullptr;
  sadi::BatchInst* d_all_scratch = nullptr;
  std::vector<sadi::BatchInst> h_all, h_all_scratch;
  // Work lists: every FFT-path group with M <= kWorkListMaxM takes each phase of the step in
  // one launch shared with the other such groups (schedule 1); schedule 0 launches every
  // group separately.  The tuner picks the schedule.
  int schedule = 1;
  sadi::WorkItem* d_items[3] = {nullptr, nullptr, nullptr};
  int n_items[3] = {0, 0, 0};
  size_t items_cap = 0;
  std::vector<char> in_list;                  // per group: covered by the work lists
  double ms_schedule[2] = {-1.0, -1.0};       // tuned ms per step of each schedule
  std::vector<void*> allocs;
  bool use_graph = false;
  hipGraphExec_t pair_exec = nullptr;         // two steps n >= 1 of a run (both buffer parities)
  long long device_bytes = 0;

  sadi_status alloc(void** p, size_t bytes) {
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
      *p = nullptr;
      return fail(SADI_E_NOMEM, std::string("hipMalloc(") + std::to_string(bytes) + "): " + hipGetErrorString(e));
    }
    allocs.push_back(*p);
    device_bytes += (long long)bytes;
    return SADI_OK;
  }
  void drop_graph() {
    if (pair_exec) (void)hipGraphExecDestroy(pair_exec);
    pair_exec = nullptr;
  }
};

namespace {

bool batch_ok(const sadi_batch* b) { return b != nullptr && b->magic == 0x5AD2; }

template <int M> struct BRowsFwd {
  static void run(const sadi_batch* b, const Group& g, const sadi::BatchInst* bi, int lf, int iu, int ip) {
    const sadi_ctx* c = b->ctx[g.members[0]];
    sadi::launch_batch_rows_fwd<M>(lf, bi, (int)g.members.size(), iu, ip, c->ldX, c->ldS, g.n, tables(c), b->stream);
  }
};
template <int M> struct BColsConv {
  static void run(const sadi_batch* b, const Group& g, const sadi::BatchInst* bi) {
    const sadi_ctx* c = b->ctx[g.members[0]];
    sadi::launch_batch_cols_conv<M>(bi, (int)g.members.size(), c->ldS, g.n, c->ldlam, tables(c), b->stream);
  }
};
template <int M> struct BRowsRhs {
  static void run(const sadi_batch* b, const Group& g, const sadi::BatchInst* bi, int mode, int iu) {
    const sadi_ctx* c = b->ctx[g.members[0]];
    sadi::launch_batch_rows_rhs<M>(mode, bi, (int)g.members.size(), iu, c->ldS, c->ldX, g.n, tables(c), b->stream);
  }
};
template <int M> struct BColsGSFwd {
  static void run(const sadi_batch* b, const Group& g, const sadi::BatchInst* bi, int ic, int ip) {
    const sadi_ctx* c = b->ctx[g.members[0]];
    sadi::launch_batch_cols_gs_fwd<M>(bi, (int)g.members.size(), ic, ip, c->ldX, c->ldS, g.n, tables(c), b->stream);
  }
};
template <int M> struct BColsGS {
  static void run(const sadi_batch* b, const Group& g, const sadi::BatchInst* bi) {
    const sadi_ctx* c = b->ctx[g.members[0]];
    sadi::launch_batch_cols_gs<M>(bi, (int)g.members.size(), c->ldX, g.n, tables(c), b->stream);
  }
};

// the two sweeps X <- H^-1 B H^-1 by dense products on the matrix cores.  Row k of the
// stored inverse is H^-1 e_k, so Hinv[k][j] = (H^-1)[j][k]: the x-sweep of every row of B is
// T = B Hinv, the y-sweep of every column of T is X[i][c] = sum_k (H^-1)[i][k] T[k][c], i.e.
// A(i, k) = Hinv[k][i] (column-contiguous A)
sadi_status dense_sweeps(sadi_batch* b, const Group& g) {
  const sadi_ctx* c = b->ctx[g.members[0]];
  const int n = g.n, cnt = (int)g.members.size();
  const int tile = g.tile[SADI_PATH_DENSE];
  sadi::launch_dgemm(n, n, n, sadi::GemmPtrs{}, g.d_prod1, cnt, true, c->ldX, n, c->ldX, 1.0, 0.0, b->stream, tile);
  sadi::launch_dgemm(n, n, n, sadi::GemmPtrs{}, g.d_prod2, cnt, false, n, c->ldX, c->ldX, 1.0, 0.0, b->stream, tile);
  return check_launch();
}

// The same sweeps with FP32 products and one FP64 refinement (B in X on entry, Uhat on exit):
//   Y = H^-1 fl32(B) H^-1 in FP32 products (FP64 result),  R = B - H Y H in FP64,
//   Uhat = Y + H^-1 fl32(R) H^-1 in FP32 products accumulated into Y.
// The FP32 solve has relative error ~ 1e-7 cond(H); after the correction it is that squared.
sadi_status mixed_sweeps(sadi_batch* b, const Group& g) {
  const sadi_ctx* c = b->ctx[g.members[0]];
  const int n = g.n, cnt = (int)g.members.size();
  const int tile = g.tile[SADI_PATH_DENSE_MIXED];
  const long ldx = c->ldX;
  for (int pass = 0; pass < 2; ++pass) {
    sadi::launch_to_fp32(g.d_cvt, cnt, n, ldx, b->stream);                                   // X32 = fl32(X)
    sadi::launch_sgemm(n, n, n, g.d_m1, cnt, true, n, n, n, 1.0, 0.0, b->stream, tile);     // T32 = X32 Hinv
    sadi::launch_sgemm(n, n, n, g.d_m2, cnt, false, n, n, n, 1.0, pass ? 1.0 : 0.0, b->stream, tile);  // Y (+)= Hinv T32
    if (pass == 0) {
      sadi::launch_dgemm(n, n, n, sadi::GemmPtrs{}, g.d_w, cnt, true, n, n, n, 1.0, 0.0, b->stream, tile);    // W = Y H
      sadi::launch_dgemm(n, n, n, sadi::GemmPtrs{}, g.d_r, cnt, true, n, n, ldx, -1.0, 1.0, b->stream, tile);  // X -= H W
    }
  }
  sadi::launch_copy_fp64(g.d_copy, cnt, n, n, ldx, b->stream);                                // X = Y
  return check_launch();
}

bool dense_ok(const sadi_batch* b, const Group& g) { return g.n <= b->dense_max_n; }

// The explicit H^-1 of every member of a group (rows H^-1 e_k: the line solve applied to
// the rows of an identity written on the device, on the batch's stream, in one allocation
// for the group) and the pointer triples of dense_sweeps; built on first use (the tuner or
// sadi_batch_set_path).
sadi_status setup_dense(sadi_batch* b, Group& g) {
  if (g.dense_ready || !dense_ok(b, g)) return SADI_OK;
  const size_t cnt = g.members.size(), nn = (size_t)g.n * g.n;
  sadi_status st;
  double* pool = nullptr;
  if ((st = b->alloc((void**)&pool, sizeof(double) * nn * cnt)) != SADI_OK) return st;
  std::vector<double*> hinv(cnt);
  std::vector<sadi::GemmPtrs> p1(cnt), p2(cnt);
  for (size_t k = 0; k < cnt; ++k) {
    sadi_ctx* c = b->ctx[g.members[k]];
    hinv[k] = pool + nn * k;
    sadi::launch_identity(hinv[k], g.n, b->stream);
    if ((st = sadi_toeplitz_solve(c, hinv[k], g.n, g.n)) != SADI_OK) return st;
    double* t = reinterpret_cast<double*>(c->S);   // N x ldX doubles fit in the spectrum buffer
    p1[k] = sadi::GemmPtrs{c->X, hinv[k], t};
    p2[k] = sadi::GemmPtrs{hinv[k], t, c->X};
  }
  const size_t pb = sizeof(sadi::GemmPtrs) * cnt;
  if ((st = b->alloc((void**)&g.d_prod1, pb)) != SADI_OK || (st = b->alloc((void**)&g.d_prod2, pb)) != SADI_OK)
    return st;
  if (hipMemcpy(g.d_prod1, p1.data(), pb, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(g.d_prod2, p2.data(), pb, hipMemcpyHostToDevice) != hipSuccess)
    return fail(SADI_E_DEVICE, "hipMemcpy");
  g.hinv.swap(hinv);
  g.dense_ready = true;
  return check_launch();
}

// Data of SADI_PATH_DENSE_MIXED for a group with explicit inverses, built on first use (the
// tuner or sadi_batch_set_path): H^-1 rounded to FP32, H itself in FP64 (from its first
// column, formed on the host exactly as the line tables' generating column), and the
// pointer arrays of mixed_sweeps.
sadi_status setup_mixed(sadi_batch* b, Group& g) {
  if (g.mixed_ready || !dense_ok(b, g)) return SADI_OK;
  sadi_status st0 = setup_dense(b, g);
  if (st0 != SADI_OK) return st0;
  const size_t cnt = g.members.size(), nn = (size_t)g.n * g.n;
  sadi_status st;
  float* pool32 = nullptr;
  double* hpool = nullptr;
  double* tcols = nullptr;
  if ((st = b->alloc((void**)&pool32, sizeof(float) * nn * cnt)) != SADI_OK ||
      (st = b->alloc((void**)&hpool, sizeof(double) * nn * cnt)) != SADI_OK ||
      (st = b->alloc((void**)&tcols, sizeof(double) * (size_t)g.n * cnt)) != SADI_OK)
    return st;
  std::vector<double> th((size_t)g.n * cnt);
  std::vector<sadi::GemmPtrs32<float>> m1(cnt);
  std::vector<sadi::GemmPtrs32<double>> m2(cnt);
  std::vector<sadi::GemmPtrs> pw(cnt), pr(cnt);
  std::vector<sadi::CvtPtrs> cv(cnt), cv_inv(cnt);
  std::vector<sadi::CopyPtrs> cp(cnt);
  std::vector<sadi::ToeplitzPtrs> tp(cnt);
  for (size_t k = 0; k < cnt; ++k) {
    sadi_ctx* c = b->ctx[g.members[k]];
    const std::vector<double> a1 = sadi::riesz_coeffs(c->alpha, g.n);
    for (int q = 0; q < g.n; ++q)
      th[k * g.n + q] = (double)((q == 0 ? 1.0L : 0.0L) + (long double)c->beta * a1[q]);
    float* hinv32 = pool32 + nn * k;
    double* hm = hpool + nn * k;
    float* x32 = reinterpret_cast<float*>(c->S);
    float* t32 = x32 + nn;
    double* w = reinterpret_cast<double*>(c->S);   // over X32 and T32 once they are consumed
    double* y = w + nn;
    cv_inv[k] = sadi::CvtPtrs{g.hinv[k], hinv32};
    tp[k] = sadi::ToeplitzPtrs{tcols + (size_t)g.n * k, hm};
    m1[k] = sadi::GemmPtrs32<float>{x32, hinv32, t32};
    m2[k] = sadi::GemmPtrs32<double>{hinv32, t32, y};
    pw[k] = sadi::GemmPtrs{y, hm, w};
    pr[k] = sadi::GemmPtrs{hm, w, c->X};
    cv[k] = sadi::CvtPtrs{c->X, x32};
    cp[k] = sadi::CopyPtrs{y, c->X};
  }
  auto upload = [&](auto** dst, const auto& v) -> sadi_status {
    const size_t bytes = sizeof(v[0]) * v.size();
    sadi_status s2 = b->alloc((void**)dst, bytes);
    if (s2 != SADI_OK) return s2;
    if (hipMemcpy(*dst, v.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) return fail(SADI_E_DEVICE, "hipMemcpy");
    return SADI_OK;
  };
  sadi::CvtPtrs* d_cv_inv = nullptr;
  sadi::ToeplitzPtrs* d_tp = nullptr;
  if ((st = upload(&g.d_m1, m1)) != SADI_OK || (st = upload(&g.d_m2, m2)) != SADI_OK ||
      (st = upload(&g.d_w, pw)) != SADI_OK || (st = upload(&g.d_r, pr)) != SADI_OK ||
      (st = upload(&g.d_cvt, cv)) != SADI_OK || (st = upload(&g.d_copy, cp)) != SADI_OK ||
      (st = upload(&d_cv_inv, cv_inv)) != SADI_OK || (st = upload(&d_tp, tp)) != SADI_OK)
    return st;
  if (hipMemcpy(tcols, th.data(), sizeof(double) * th.size(), hipMemcpyHostToDevice) != hipSuccess)
    return fail(SADI_E_DEVICE, "hipMemcpy");
  sadi::launch_to_fp32(d_cv_inv, (int)cnt, g.n, g.n, b->stream);
  sadi::launch_toeplitz_fill(d_tp, (int)cnt, g.n, b->stream);
  g.mixed_ready = true;
  return check_launch();
}

bool wl_eligible(const Group& g) { return g.path == SADI_PATH_FFT_GS && g.m <= sadi::kWorkListMaxM; }

// The three work lists of the current paths.  Whole instances are spread over the 8 XCDs by
// cost (largest first to the least loaded), so that the column groups of one instance share
// that XCD's L2; dispatch sends slot 8 q + x to XCD x, so slot 8 q + x holds the q-th item of
// XCD x's list (empty items pad the shorter lists).
sadi_status build_worklists(sadi_batch* b) {
  b->in_list.assign(b->groups.size(), 0);
  for (int ph = 0; ph < 3; ++ph) b->n_items[ph] = 0;
  if (b->schedule == 0) return SADI_OK;
  for (size_t gi = 0; gi < b->groups.size(); ++gi) b->in_list[gi] = wl_eligible(b->groups[gi]) ? 1 : 0;
  for (int ph = 0; ph < 3; ++ph) {
    struct Inst {
      int idx, blocks;
      double cost;
    };
    std::vector<Inst> insts;
    for (size_t gi = 0; gi < b->groups.size(); ++gi) {
      if (!b->in_list[gi]) continue;
      const Group& g = b->groups[gi];
      int blocks[3];
      double cost[3];
      sadi::worklist_shape(g.m, g.n, blocks, cost);
      for (int i : g.members) insts.push_back(Inst{i, blocks[ph], blocks[ph] * cost[ph]});
    }
    if (insts.empty()) continue;
    std::stable_sort(insts.begin(), insts.end(), [](const Inst& a, const Inst& c) { return a.cost > c.cost; });
    std::vector<std::vector<sadi::WorkItem>> xcd(8);
    double load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (const Inst& in : insts) {
      const int x = (int)(std::min_element(load, load + 8) - load);
      load[x] += in.cost;
      for (int blk = 0; blk < in.blocks; ++blk) xcd[x].push_back(sadi::WorkItem{in.idx, blk});
    }
    size_t len = 0;
    for (auto& v : xcd) len = std::max(len, v.size());
    std::vector<sadi::WorkItem> items(8 * len, sadi::WorkItem{-1, 0});
    for (size_t q = 0; q < len; ++q)
      for (int x = 0; x < 8; ++x)
        if (q < xcd[x].size()) items[8 * q + x] = xcd[x][q];
    if (items.size() > b->items_cap) {
      for (int p = 0; p < 3; ++p) {
        if (b->d_items[p]) (void)hipFree(b->d_items[p]);
        b->d_items[p] = nullptr;
      }
      b->items_cap = 0;
      for (int p = 0; p < 3; ++p) {
        void* q = nullptr;
        if (hipMalloc(&q, sizeof(sadi::WorkItem) * items.size()) != hipSuccess)
          return fail(SADI_E_NOMEM, "work list allocation");
        b->d_items[p] = (sadi::WorkItem*)q;
      }
      b->items_cap = items.size();
      // the lists of the other phases are rebuilt below
      for (int p = 0; p < ph; ++p) b->n_items[p] = 0;
      return build_worklists(b);
    }
    SADI_HIP(hipMemcpy(b->d_items[ph], items.data(), sizeof(sadi::WorkItem) * items.size(), hipMemcpyHostToDevice));
    b->n_items[ph] = (int)items.size();
  }
  return SADI_OK;
}

// one step of every group.  first: start-up step (x0 = u[iu], phi2); otherwise lf selects
// the deferred update in the row transform (u[ip] <- 2 u[iu] - u[ip] + X, then the step
// advances u[ip]).  On return X holds each instance's increment.
// One step for every group.  first: the start-up step (four kernels, the increment left in
// X).  Otherwise, in a run: dense groups take the four-kernel step whose row pass first
// applies the previous step's deferred update (lf); FFT groups take three kernels on a
// grid whose orientation alternates, the state u[su] advanced into u[so] (transposed), and
// the row transform already in S from the run's start or the step before.
sadi_status batch_step(sadi_batch* b, bool scratch, bool first, int lf, int iu, int ip) {
  const int su = lf ? ip : iu;   // the state this step advances
  const bool lists = !first && b->in_list.size() == b->groups.size();
  if (lists && (b->n_items[0] > 0 || b->n_items[1] > 0 || b->n_items[2] > 0)) {
    const sadi::BatchInst* all = scratch ? b->d_all_scratch : b->d_all;
    for (int ph = 0; ph < 3; ++ph)
      sadi::launch_worklist(ph, all, b->d_items[ph], b->n_items[ph], su, 1 - su, b->stream);
  }
  for (size_t gi = 0; gi < b->groups.size(); ++gi) {
    Group& g = b->groups[gi];
    if (lists && b->in_list[gi]) continue;   // done by the work lists
    const sadi::BatchInst* bi = scratch ? g.d_scratch_inst : g.d_inst;
    if (!first && g.path == SADI_PATH_FFT_GS) {
      dispatch_m<BColsConv>(g.m, b, g, bi);
      dispatch_m<BRowsRhs>(g.m, b, g, bi, 0, su);
      dispatch_m<BColsGSFwd>(g.m, b, g, bi, su, 1 - su);
      continue;
    }
    dispatch_m<BRowsFwd>(g.m, b, g, bi, lf, iu, ip);
    dispatch_m<BColsConv>(g.m, b, g, bi);
    if (g.path == SADI_PATH_FFT_GS) {
      dispatch_m<BRowsRhs>(g.m, b, g, bi, first ? 1 : 0, su);
      dispatch_m<BColsGS>(g.m, b, g, bi);
    } else {
      dispatch_m<BRowsRhs>(g.m, b, g, bi, first ? 4 : 3, su);
      sadi_status st = g.path == SADI_PATH_DENSE ? dense_sweeps(b, g) : mixed_sweeps(b, g);
      if (st != SADI_OK) return st;
    }
  }
  return check_launch();
}

sadi_status batch_leapfrog(sadi_batch* b, bool scratch, int mode, int ic, int ip, bool fft_groups_too = true) {
  for (Group& g : b->groups) {
    if (!fft_groups_too && g.path == SADI_PATH_FFT_GS) continue;
    const sadi_ctx* c = b->ctx[g.members[0]];
    sadi::launch_batch_leapfrog(mode, scratch ? g.d_scratch_inst : g.d_inst, (int)g.members.size(), ic, ip, c->ldX,
                                g.n, b->stream);
  }
  return check_launch();
}

// nsteps steps n >= 1 from (u[0], u[1]) = (u^{n-1}, u^n); the result is left the same way
sadi_status batch_run(sadi_batch* b, bool scratch, int nsteps, bool graph) {
  if (nsteps <= 0) return SADI_OK;
  // FFT groups: u^{n-1} into the transposed layout, the row transform of u^n into S
  for (Group& g : b->groups) {
    if (g.path != SADI_PATH_FFT_GS) continue;
    const sadi::BatchInst* bi = scratch ? g.d_scratch_inst : g.d_inst;
    sadi::launch_batch_transpose(bi, (int)g.members.size(), 0, g.n, b->stream);
    dispatch_m<BRowsFwd>(g.m, b, g, bi, 0, 1, 0);
  }
  sadi_status st = batch_step(b, scratch, false, 0, 1, 0);
  if (st != SADI_OK) return st;
  int cur = 1, prev = 0;
  int left = nsteps - 1;
  if (graph && !scratch && left >= 2) {
    if (!b->pair_exec) {
      // capture two steps (cur = 1, then cur = 0): the buffer roles repeat every two steps
      hipGraph_t gr = nullptr;
      SADI_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
      sadi_status s1 = batch_step(b, false, false, 1, 1, 0);
      sadi_status s2 = s1 == SADI_OK ? batch_step(b, false, false, 1, 0, 1) : s1;
      hipError_t e = hipStreamEndCapture(b->stream, &gr);
      if (s2 != SADI_OK) {
        if (gr) (void)hipGraphDestroy(gr);
        return s2;
      }
      if (e != hipSuccess) return fail(SADI_E_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
      e = hipGraphInstantiate(&b->pair_exec, gr, nullptr, nullptr, 0);
      (void)hipGraphDestroy(gr);
      if (e != hipSuccess) {
        b->pair_exec = nullptr;
        return fail(SADI_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
      }
    }
    for (; left >= 2; left -= 2) SADI_HIP(hipGraphLaunch(b->pair_exec, b->stream));
  }
  for (; left > 0; --left) {
    st = batch_step(b, scratch, false, 1, cur, prev);
    if (st != SADI_OK) return st;
    std::swap(cur, prev);
  }
  // FFT groups: the newest state is in u[prev] (transposed when nsteps is odd), the one
  // before in u[cur]; both go back to the natural layout with the newest in u[1]
  for (Group& g : b->groups) {
    if (g.path != SADI_PATH_FFT_GS) continue;
    const sadi::BatchInst* bi = scratch ? g.d_scratch_inst : g.d_inst;
    if (prev == 1)
      sadi::launch_batch_transpose(bi, (int)g.members.size(), 0, g.n, b->stream);
    else
      sadi::launch_batch_swap_transposed(bi, (int)g.members.size(), g.n, b->stream);
  }
  // dense groups: pending newest = 2 u[cur] - u[prev] + X; leave it in u[1], the step before
  // in u[0]
  return cur == 1 ? batch_leapfrog(b, scratch, 2, 1, 0, false) : batch_leapfrog(b, scratch, 0, 0, 1, false);
}

sadi_status upload_desc(sadi_batch* b, Group& g, bool scratch, const std::vector<double*>& s0,
                        const std::vector<double*>& s1) {
  std::vector<sadi::BatchInst> h(g.members.size());
  for (size_t k = 0; k < g.members.size(); ++k) {
    const int i = g.members[k];
    const sadi_ctx* c = b->ctx[i];
    sadi::BatchInst& d = h[k];
    d.u[0] = s0[k];
    d.u[1] = s1[k];
    d.phi2 = scratch ? s0[k] : b->phi2[i];
    d.S = c->S;
    d.X = c->X;
    d.lam2d = c->lam2d;
    d.lam_s = c->lam_s;
    d.lam_c = c->lam_c;
    d.f = c->f;
    d.r = c->r;
    d.sc = scalars(c, false);
    d.n = c->n;
    d.m = c->m;
    d.lds = c->ldS;
    d.ldx = c->ldX;
    d.ldlam = c->ldlam;
    d.tab = tables(c);
    (scratch ? b->h_all_scratch : b->h_all)[i] = d;
  }
  sadi::BatchInst* dst = scratch ? g.d_scratch_inst : g.d_inst;
  SADI_HIP(hipMemcpy(dst, h.data(), sizeof(sadi::BatchInst) * h.size(), hipMemcpyHostToDevice));
  return SADI_OK;
}

// the descriptor array of all instances (after upload_desc of every group)
sadi_status upload_all(sadi_batch* b, bool scratch) {
  const std::vector<sadi::BatchInst>& h = scratch ? b->h_all_scratch : b->h_all;
  SADI_HIP(hipMemcpy(scratch ? b->d_all_scratch : b->d_all, h.data(), sizeof(sadi::BatchInst) * h.size(),
                     hipMemcpyHostToDevice));
  return SADI_OK;
}

// start-up step uses the scalars of the first step (w = 1/2); they differ only by that factor
sadi_status set_scalars(sadi_batch* b, Group& g, bool first) {
  std::vector<sadi::BatchInst> h(g.members.size());
  SADI_HIP(hipMemcpy(h.data(), g.d_inst, sizeof(sadi::BatchInst) * h.size(), hipMemcpyDeviceToHost));
  for (size_t k = 0; k < g.members.size(); ++k) {
    h[k].sc = scalars(b->ctx[g.members[k]], first);
    b->h_all[g.members[k]].sc = h[k].sc;
  }
  SADI_HIP(hipMemcpy(g.d_inst, h.data(), sizeof(sadi::BatchInst) * h.size(), hipMemcpyHostToDevice));
  return SADI_OK;
}

void destroy_batch(sadi_batch* b) {
  b->drop_graph();
  for (int p = 0; p < 3; ++p)
    if (b->d_items[p]) (void)hipFree(b->d_items[p]);
  for (void* p : b->allocs) (void)hipFree(p);
  for (sadi_ctx* c : b->ctx)
    if (c) (void)sadi_destroy(c);
  if (b->own_stream) (void)hipStreamDestroy(b->own_stream);
  b->magic = 0;
  delete b;
}

}  // namespace

extern "C" {

sadi_status sadi_batch_create(int count, const int* n, const double* alpha, const double* kappa, double tau,
                              const double* domain, int dense_max_n, sadi_batch** out) {
  if (!out) return fail(SADI_E_INVALID, "out is NULL");
  *out = nullptr;
  if (count <= 0) return fail(SADI_E_INVALID, "count must be positive");
  if (!n || !alpha || !kappa || !domain) return fail(SADI_E_INVALID, "NULL array");
  for (int i = 0; i < count; ++i) {
    sadi_status st = validate_problem(alpha[i], kappa[i], n[i], tau, domain, false);
    if (st != SADI_OK) return fail(st, std::string("instance ") + std::to_string(i) + ": " + sadi_last_error());
  }
  sadi_batch* b = new (std::nothrow) sadi_batch;
  if (!b) return fail(SADI_E_NOMEM, "host allocation");
  auto bail = [&](sadi_status st) {
    const std::string msg = sadi_last_error();
    destroy_batch(b);
    return fail(st, msg);
  };
  b->count = count;
  b->dense_max_n = dense_max_n;
  b->ctx.assign(count, nullptr);
  {
    // instances set up concurrently, one host thread each
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const int workers = (int)std::min<unsigned>(std::min<unsigned>(hw, 16u), (unsigned)count);
    const int inner = 1;
    std::vector<sadi_status> status(count, SADI_OK);
    std::vector<std::string> errors(count);
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) device = 0;
    std::vector<std::thread> pool;
    for (int w = 0; w < workers; ++w)
      pool.emplace_back([&, w] {
        (void)hipSetDevice(device);   // the caller's device, as for sadi_setup
        g_setup_threads = inner;
        g_setup_no_run_state = true;   // batch members take batched steps only
        g_setup_defer_gs = true;       // their line tables: one launch for all, below
        for (int i = w; i < count; i += workers) {
          status[i] = sadi_setup(alpha[i], kappa[i], n[i], tau, domain, &b->ctx[i]);
          if (status[i] != SADI_OK) errors[i] = sadi_last_error();
        }
      });
    for (auto& th : pool) th.join();
    for (int i = 0; i < count; ++i)
      if (status[i] != SADI_OK) {
        const std::string msg = std::string("instance ") + std::to_string(i) + ": " + errors[i];
        destroy_batch(b);
        return fail(status[i], msg);
      }
  }
  if (hipStreamCreate(&b->own_stream) != hipSuccess) {
    b->own_stream = nullptr;
    return bail(fail(SADI_E_DEVICE, "hipStreamCreate"));
  }
  b->stream = b->own_stream;
  for (sadi_ctx* c : b->ctx) c->stream = b->stream;
  {
    // the members' line tables (Levinson recursion and tables, one workgroup per member)
    std::vector<sadi::GsJob> jobs;
    int max_m = 0;
    for (sadi_ctx* c : b->ctx)
      if (c->gs_pending) {
        jobs.push_back(c->gs_job);
        max_m = std::max(max_m, c->gs_job.m);
      }
    if (!jobs.empty()) {
      void* dj = nullptr;
      if (hipMalloc(&dj, sizeof(sadi::GsJob) * jobs.size()) != hipSuccess)
        return bail(fail(SADI_E_NOMEM, "line table jobs"));
      hipError_t e = hipMemcpy(dj, jobs.data(), sizeof(sadi::GsJob) * jobs.size(), hipMemcpyHostToDevice);
      if (e == hipSuccess) {
        sadi::launch_gs_generator_batched((const sadi::GsJob*)dj, (int)jobs.size(), max_m, b->stream);
        e = hipGetLastError();
      }
      if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
      (void)hipFree(dj);
      if (e != hipSuccess) return bail(fail(SADI_E_DEVICE, std::string("line tables: ") + hipGetErrorString(e)));
      for (sadi_ctx* c : b->ctx) c->gs_pending = false;
    }
  }

  std::map<int, int> by_n;
  for (int i = 0; i < count; ++i) {
    auto it = by_n.find(n[i]);
    if (it == by_n.end()) {
      by_n[n[i]] = (int)b->groups.size();
      Group g;
      g.n = n[i];
      g.m = b->ctx[i]->m;
      b->groups.push_back(g);
      b->groups.back().members.push_back(i);
    } else {
      b->groups[it->second].members.push_back(i);
    }
  }
  {
    sadi_status st;
    if ((st = b->alloc((void**)&b->d_all, sizeof(sadi::BatchInst) * count)) != SADI_OK ||
        (st = b->alloc((void**)&b->d_all_scratch, sizeof(sadi::BatchInst) * count)) != SADI_OK)
      return bail(st);
    b->h_all.assign(count, sadi::BatchInst{});
    b->h_all_scratch.assign(count, sadi::BatchInst{});
  }
  for (Group& g : b->groups) {
    const size_t cnt = g.members.size();
    sadi_status st;
    if ((st = b->alloc((void**)&g.d_inst, sizeof(sadi::BatchInst) * cnt)) != SADI_OK) return bail(st);
    if ((st = b->alloc((void**)&g.d_scratch_inst, sizeof(sadi::BatchInst) * cnt)) != SADI_OK) return bail(st);
  }
  if (hipStreamSynchronize(b->stream) != hipSuccess) return bail(fail(SADI_E_DEVICE, "setup synchronisation"));
  *out = b;
  return SADI_OK;
}

sadi_status sadi_batch_bind(sadi_batch* b, double* const* u_prev, double* const* u_cur, const double* const* phi2) {
  if (!batch_ok(b)) return fail(SADI_E_STATE, "invalid batch");
  if (!u_prev || !u_cur) return fail(SADI_E_INVALID, "NULL array");
  for (int i = 0; i < b->count; ++i) {
    if (!u_prev[i] || !u_cur[i]) return fail(SADI_E_INVALID, "NULL state pointer for instance " + std::to_string(i));
    if (u_prev[i] == u_cur[i]) return fail(SADI_E_INVALID, "u_prev and u_cur alias for instance " + std::to_string(i));
  }
  b->u_prev.assign(u_prev, u_prev + b->count);
  b->u_cur.assign(u_cur, u_cur + b->count);
  b->phi2.assign(b->count, nullptr);
  if (phi2)
    for (int i = 0; i < b->count; ++i) b->phi2[i] = phi2[i];
  for (Group& g : b->groups) {
    std::vector<double*> s0, s1;
    for (int i : g.members) {
      s0.push_back(b->u_prev[i]);
      s1.push_back(b->u_cur[i]);
    }
    sadi_status st = upload_desc(b, g, false, s0, s1);
    if (st != SADI_OK) return st;
  }
  sadi_status st = upload_all(b, false);
  if (st == SADI_OK) st = build_worklists(b);
  if (st != SADI_OK) return st;
  b->drop_graph();
  b->bound = true;
  return SADI_OK;
}

sadi_status sadi_batch_first_step(sadi_batch* b) {
  if (!batch_ok(b)) return fail(SADI_E_STATE, "invalid batch");
  if (!b->bound) return fail(SADI_E_STATE, "no state bound");
  for (int i = 0; i < b->count; ++i)
    if (!b->phi2[i]) return fail(SADI_E_INVALID, "no phi2 bound for instance " + std::to_string(i));
  for (Group& g : b->groups) {
    sadi_status st = set_scalars(b, g, true);
    if (st != SADI_OK) return st;
  }
  sadi_status st = batch_step(b, false, true, 0, 0, 1);
  if (st == SADI_OK) st = batch_leapfrog(b, false, 1, 0, 1);
  for (Group& g : b->groups) {
    sadi_status s2 = set_scalars(b, g, false);
    if (st == SADI_OK) st = s2;
  }
  if (st == SADI_OK) st = upload_all(b, false);
  return st;
}

sadi_status sadi_batch_run(sadi_batch* b, int nsteps) {
  if (!batch_ok(b)) return fail(SADI_E_STATE, "invalid batch");
  if (!b->bound) return fail(SADI_E_STATE, "no state bound");
  if (nsteps < 0) return fail(SADI_E_INVALID, "nsteps must be >= 0");
  return batch_run(b, false, nsteps, b->use_graph);
}

sadi_status sadi_batch_set_graph(sadi_batch* b, int enable) {
  if (!batch_ok(b)) return fail(SADI_E_STATE, "invalid batch");
  b->use_graph = enable != 0;
  if (!b->use_graph) b->drop_graph();
  return SADI_OK;
}

sadi_status sadi_batch_set_path(sadi_batch* b, int n, int path) {
  if (!batch_ok(b)) return fail(SADI_E_STATE, "invalid batch");
  if (path != SADI_PATH_FFT_GS && !dense_path(path)) return fail(SADI_E_INVALID, "unknown path");
  for (Group& g : b->groups) {
    if (g.n != n) continue;
    if (dense_path(path) && !dense_ok(b, g))
      return fail(SADI_E_UNSUPPORTED, "no explicit inverse for N = " + std::to_string(n) + " (above dense_max_n)");
    if (dense_path(path)) {
      const sadi_status st = path == SADI_PATH_DENSE ? setup_dense(b, g) : setup_mixed(b, g);
      if (st != SADI_OK) return st;
    }
    g.path = path;
    b->drop_graph();
    return b->bound ? build_worklists(b) : SADI_OK;
  }
  return fail(SADI_E_INVALID, "no instance with N = " + std::to_string(n));
}

sadi_status sadi_batch_tune(sadi_batch* b, int steps) {
  if (!batch_ok(b)) return fail(SADI_E_STATE, "invalid batch");
  if (steps < 1) return fail(SADI_E_INVALID, "steps must be >= 1");
  // scratch state (zeros) so that the caller's state is untouched
  std::vector<void*> tmp;
  auto cleanup = [&]() {
    for (void* p : tmp) (void)hipFree(p);
  };
  for (Group& g : b->groups) {
    std::vector<double*> s0, s1;
    for (size_t k = 0; k < g.members.size(); ++k) {
      void* p0 = nullptr;
      void* p1 = nullptr;
      const size_t bytes = sizeof(double) * (size_t)g.n * g.n;
      if (hipMalloc(&p0, bytes) != hipSuccess || hipMalloc(&p1, bytes) != hipSuccess) {
        if (p0) (void)hipFree(p0);
        cleanup();
        return fail(SADI_E_NOMEM, "tuning scratch state");
      }
      tmp.push_back(p0);
      tmp.push_back(p1);
      (void)hipMemset(p0, 0, bytes);
      (void)hipMemset(p1, 0, bytes);
      s0.push_back((double*)p0);
      s1.push_back((double*)p1);
    }
    sadi_status st = upload_desc(b, g, true, s0, s1);
    if (st != SADI_OK) {
      cleanup();
      return st;
    }
  }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    cleanup();
    return fail(SADI_E_DEVICE, "hipEventCreate");
  }
  for (Group& g : b->groups) g.ms[0] = g.ms[1] = g.ms[2] = -1.0;
  const std::vector<int> saved = [&] {
    std::vector<int> v;
    for (Group& g : b->groups) v.push_back(g.path);
    return v;
  }();
  sadi_status st = SADI_OK;
  const int saved_schedule = b->schedule;
  b->schedule = 0;   // groups timed alone launch separately
  if ((st = build_worklists(b)) != SADI_OK || (st = upload_all(b, true)) != SADI_OK) {
    b->schedule = saved_schedule;
    cleanup();
    return st;
  }
  // time each group alone: the other groups are skipped by moving them out temporarily
  std::vector<Group> all;
  all.swap(b->groups);
  for (size_t gi = 0; gi < all.size() && st == SADI_OK; ++gi) {
    if ((st = setup_mixed(b, all[gi])) != SADI_OK) break;
    b->groups.assign(1, all[gi]);
    // the Gohberg-Semencul path, then both dense paths with each tile shape of their products
    const int variants[5][2] = {{SADI_PATH_FFT_GS, 0},      {SADI_PATH_DENSE, 64},      {SADI_PATH_DENSE, 32},
                                {SADI_PATH_DENSE_MIXED, 64}, {SADI_PATH_DENSE_MIXED, 32}};
    for (int v = 0; v < 5 && st == SADI_OK; ++v) {
      const int path = variants[v][0];
      if (dense_path(path) && !dense_ok(b, all[gi])) continue;
      b->groups[0].path = path;
      b->groups[0].tile[path] = variants[v][1];
      st = batch_run(b, true, 2, false);   // warm-up
      if (st != SADI_OK) break;
      (void)hipEventRecord(e0, b->stream);
      st = batch_run(b, true, steps, false);
      (void)hipEventRecord(e1, b->stream);
      if (hipEventSynchronize(e1) != hipSuccess) st = fail(SADI_E_DEVICE, "tuning run");
      float ms = 0.0f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      const double per = ms / steps;
      if (all[gi].ms[path] < 0.0 || per < all[gi].ms[path]) {
        all[gi].ms[path] = per;
        all[gi].tile[path] = variants[v][1];
      }
    }
    b->groups.clear();
  }
  b->groups.swap(all);
  for (size_t gi = 0; gi < b->groups.size(); ++gi) {
    Group& g = b->groups[gi];
    g.path = saved[gi];
    if (st == SADI_OK) {
      g.path = SADI_PATH_FFT_GS;
      for (int p : {SADI_PATH_DENSE, SADI_PATH_DENSE_MIXED})
        if (g.ms[p] >= 0.0 && g.ms[p] < g.ms[g.path]) g.path = p;
    }
  }
  // then the schedule of the whole step with those paths: every group on its own, or the
  // FFT groups up to kWorkListMaxM sharing one launch per phase
  b->schedule = saved_schedule;
  for (int sched = 0; sched < 2 && st == SADI_OK; ++sched) {
    b->schedule = sched;
    if ((st = build_worklists(b)) != SADI_OK) break;
    if ((st = batch_run(b, true, 2, false)) != SADI_OK) break;
    (void)hipEventRecord(e0, b->stream);
    st = batch_run(b, true, steps, false);
    (void)hipEventRecord(e1, b->stream);
    if (hipEventSynchronize(e1) != hipSuccess) st = fail(SADI_E_DEVICE, "tuning run");
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    b->ms_schedule[sched] = ms / steps;
  }
  if (st == SADI_OK) b->schedule = b->ms_schedule[1] <= b->ms_schedule[0] ? 1 : 0;
  else b->schedule = saved_schedule;
  {
    const sadi_status s2 = build_worklists(b);
    if (st == SADI_OK) st = s2;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(b->stream);
  cleanup();
  b->drop_graph();
  return st;
}

sadi_status sadi_batch_set_schedule(sadi_batch* b, int schedule) {
  if (!batch_ok(b)) return fail(SADI_E_STATE, "invalid batch");
  if (schedule != 0 && schedule != 1) return fail(SADI_E_INVALID, "schedule must be 0 or 1");
  b->schedule = schedule;
  b->drop_graph();
  return b->bound ? build_worklists(b) : SADI_OK;
}

sadi_status sadi_batch_get_schedule(const sadi_batch* b, int* schedule, double* ms_groups, double* ms_lists) {
  if (!batch_ok(b)) return fail(SADI_E_STATE, "invalid batch");
  if (schedule) *schedule = b->schedule;
  if (ms_groups) *ms_groups = b->ms_schedule[0];
  if (ms_lists) *ms_lists = b->ms_schedule[1];
  return SADI_OK;
}

sadi_status sadi_batch_get_group(const sadi_batch* b, int index, int* n, int* members, int* path, double* ms_fft,
                                 double* ms_dense, double* ms_dense_mixed, int* dense_tile) {
  if (!batch_ok(b)) return fail(SADI_E_STATE, "invalid batch");
  if (index < 0 || index >= (int)b->groups.size()) return fail(SADI_E_INVALID, "group index out of range");
  const Group& g = b->groups[index];
  if (n) *n = g.n;
  if (members) *members = (int)g.members.size();
  if (path) *path = g.path;
  if (ms_fft) *ms_fft = g.ms[SADI_PATH_FFT_GS];
  if (ms_dense) *ms_dense = g.ms[SADI_PATH_DENSE];
  if (ms_dense_mixed) *ms_dense_mixed = g.ms[SADI_PATH_DENSE_MIXED];
  if (dense_tile) *dense_tile = g.tile[g.path == SADI_PATH_DENSE_MIXED ? SADI_PATH_DENSE_MIXED : SADI_PATH_DENSE];
  return SADI_OK;
}

sadi_status sadi_batch_get_info(const sadi_batch* b, int* count, int* groups, long long* bytes) {
  if (!batch_ok(b)) return fail(SADI_E_STATE, "invalid batch");
  long long total = b->device_bytes;
  for (const sadi_ctx* c : b->ctx) total += c->device_bytes;
  if (count) *count = b->count;
  if (groups) *groups = (int)b->groups.size();
  if (bytes) *bytes = total;
  return SADI_OK;
}

sadi_status sadi_batch_synchronize(sadi_batch* b) {
  if (!batch_ok(b)) return fail(SADI_E_STATE, "invalid batch");
  SADI_HIP(hipStreamSynchronize(b->stream));
  return SADI_OK;
}

sadi_status sadi_batch_destroy(sadi_batch* b) {
  if (!batch_ok(b)) return fail(SADI_E_STATE, "invalid batch");
  (void)hipStreamSynchronize(b->stream);
  destroy_batch(b);
  return SADI_OK;
}

}  // extern "C"
