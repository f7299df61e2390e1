// Batched driver: cpca_solve_batched runs FISTA on the sampled matrix and
// the alternate decoder for many (instance, gamma) tasks at once.
//
// All tasks are resident together. Each launch covers every task through a
// block -> task table (batched.hpp); the FISTA iterations and chunks of CG
// iterations are captured once as HIP graphs and replayed, so the host only
// polls the per-task convergence flags between chunks. Finished tasks make
// their workgroups return immediately. The launch shape of the batched
// fused product comes from the autotuner (or the handle's override).
#include "batched.hpp"
#include "common.hpp"
#define CPCA_SPECTRAL_HOST
#include "spectral.hpp"

namespace {

struct InstHost {
  HostCsr Lr, Lc, Lrt, Lct;
  std::vector<uint8_t> mr, mc;  // mc padded to ld
  int64_t ld = 0, ldt = 0;
  GraphImage<double> g64{}, gt{};
  GraphImage<float> g32{};
  size_t o_zmr = 0, o_zmc = 0;
};

inline int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

cpca_status check_batched_args(cpca_mode mode, const cpca_instance* inst, int32_t ninst,
                               const cpca_task* tasks, int32_t ntasks, int32_t fista_iters,
                               double tol, int32_t max_iter) {
  STCHK(check_mode(mode));
  if (!inst || ninst < 1) return fail(CPCA_EINVAL, "batched: no instances");
  if (!tasks || ntasks < 1) return fail(CPCA_EINVAL, "batched: no tasks");
  if (fista_iters < 0) return fail(CPCA_EINVAL, "batched: fista_iters < 0");
  if (!std::isfinite(tol) || !(tol > 0)) return fail(CPCA_EINVAL, "batched: tol must be > 0");
  if (max_iter < 1) return fail(CPCA_EINVAL, "batched: max_iter < 1");
  for (int32_t k = 0; k < ninst; ++k) {
    const cpca_instance& I = inst[k];
    char where[64];
    std::snprintf(where, sizeof where, "instance %d", k);
    cpca_status st = check_decode_args(mode, I.rho_r, I.rho_c, I.omega_r, I.omega_c, I.p, I.n,
                                       I.Lr, I.Lc, 0.0, 0.0, tol, max_iter);
    if (st) return fail(st, std::string(where) + ": " + last_error());
    if ((st = check_csr_shape("Lr_til", I.Lr_til, I.rho_r)))
      return fail(st, std::string(where) + ": " + last_error());
    if ((st = check_csr_shape("Lc_til", I.Lc_til, I.rho_c)))
      return fail(st, std::string(where) + ": " + last_error());
    if (!I.Ytil) return fail(CPCA_EINVAL, std::string(where) + ": null Ytil");
    // lmax <= 0 asks the library to estimate the norm (device power iteration)
    if (!std::isfinite(I.lmax_r_til) || !std::isfinite(I.lmax_c_til))
      return fail(CPCA_EINVAL, std::string(where) + ": lmax must be finite");
  }
  for (int32_t t = 0; t < ntasks; ++t) {
    const cpca_task& T = tasks[t];
    char where[64];
    std::snprintf(where, sizeof where, "task %d", t);
    if (T.instance < 0 || T.instance >= ninst)
      return fail(CPCA_EINVAL, std::string(where) + ": instance index out of range");
    cpca_status st;
    if ((st = check_gamma("gamma_r", T.gamma_r)) || (st = check_gamma("gamma_c", T.gamma_c)))
      return fail(st, std::string(where) + ": " + last_error());
    if (!T.X_out) return fail(CPCA_EINVAL, std::string(where) + ": null X_out");
  }
  return CPCA_OK;
}

struct BatchCfg {
  int R = 1;
  bool lds = true;
};

template <typename T, int KIND>
hipError_t launch_bapply(cpca_handle h, hipStream_t s, const BatchCfg& c, int grid, size_t ld_max,
                         const BTask* tasks, const int* tab, double* part, double fc, int par) {
  constexpr int VEC = (int)(16 / sizeof(T));
  const size_t shm = c.lds ? (size_t)c.R * ld_max * sizeof(T) : 0;
  (void)h;
#define CPCA_B(RV, LV) \
  k_apply_batched<T, RV, LV, VEC, KIND><<<grid, kThreads, shm, s>>>(tasks, tab, part, fc, par)
  switch (c.R * 2 + (c.lds ? 1 : 0)) {
    case 3: CPCA_B(1, true); break;
    case 2: CPCA_B(1, false); break;
    case 5: CPCA_B(2, true); break;
    case 4: CPCA_B(2, false); break;
    case 9: CPCA_B(4, true); break;
    case 8: CPCA_B(4, false); break;
    default: return hipErrorInvalidValue;
  }
#undef CPCA_B
  return hipGetLastError();
}

struct Grids {
  int a = 0, f = 0, v = 0;  // apply / FISTA / vector block counts (for the chosen R)
};

// Block tables for rows-per-workgroup R (the apply and FISTA slices depend
// on R, the vector slices do not). With `only`, tasks whose entry is 0 get no
// blocks (their block ranges keep stale values that no block reads).
void build_tables(std::vector<BTask>& bt, int R, std::vector<int>& atab, std::vector<int>& ftab,
                  std::vector<int>& vtab, Grids& g, const std::vector<char>* only = nullptr) {
  atab.clear();
  ftab.clear();
  vtab.clear();
  for (size_t t = 0; t < bt.size(); ++t) {
    if (only && !(*only)[t]) continue;
    BTask& k = bt[t];
    k.anrb = (k.p + R - 1) / R;
    k.aper = (k.anrb + 7) / 8;
    k.ablk0 = (int)atab.size();
    atab.insert(atab.end(), 8 * k.aper, (int)t);
    k.fnrb = (k.rho_r + R - 1) / R;
    k.fper = (k.fnrb + 7) / 8;
    k.fblk0 = (int)ftab.size();
    ftab.insert(ftab.end(), 8 * k.fper, (int)t);
    const size_t nv = (size_t)k.p * k.ld / 4;
    k.nvblk = (int)std::max<size_t>(1, std::min<size_t>((nv + kThreads - 1) / kThreads, 256));
    k.vblk0 = (int)vtab.size();
    vtab.insert(vtab.end(), k.nvblk, (int)t);
  }
  g.a = (int)atab.size();
  g.f = (int)ftab.size();
  g.v = (int)vtab.size();
}

cpca_status run_batched(cpca_handle h, cpca_mode mode, const cpca_instance* inst, int32_t ninst,
                        const cpca_task* tasks, int32_t ntasks, int32_t J, double tol,
                        int32_t max_iter, cpca_info* infos) {
  const auto t0 = std::chrono::steady_clock::now();
  const bool f32 = mode != CPCA_FP64;
  HIPCHK(hipStreamSynchronize(h->stream));
  // ---- host preparation: validation of every graph and index set, images
  std::vector<InstHost> ih((size_t)ninst);
  Staging stg;
  int64_t ld_max = 0, ldt_max = 0;
  for (int32_t k = 0; k < ninst; ++k) {
    const cpca_instance& I = inst[k];
    InstHost& H = ih[(size_t)k];
    STCHK(fetch_csr("Lr", I.Lr, H.Lr));
    STCHK(fetch_csr("Lc", I.Lc, H.Lc));
    STCHK(fetch_csr("Lr_til", I.Lr_til, H.Lrt));
    STCHK(fetch_csr("Lc_til", I.Lc_til, H.Lct));
    std::vector<uint8_t> mc;
    STCHK(fetch_index_set("omega_r", I.omega_r, I.rho_r, I.p, H.mr));
    STCHK(fetch_index_set("omega_c", I.omega_c, I.rho_c, I.n, mc));
    H.ld = round_up(I.n, 4);
    H.ldt = round_up(I.rho_c, 4);
    ld_max = std::max(ld_max, H.ld);
    ldt_max = std::max(ldt_max, H.ldt);
    H.mc.assign((size_t)H.ld, 0);
    std::copy(mc.begin(), mc.end(), H.mc.begin());
    H.g64 = stage_graph<double>(stg, H.Lr, H.Lc, H.mr, H.mc, kWave * 2);
    if (f32) H.g32 = stage_graph<float>(stg, H.Lr, H.Lc, H.mr, H.mc, kWave * 4);
    std::vector<uint8_t> zr((size_t)I.rho_r, 0), zc((size_t)H.ldt, 0);
    H.gt = stage_graph<double>(stg, H.Lrt, H.Lct, zr, zc, kWave * 2);
  }
  // norms of the sampled graphs: the caller's, or estimated on the device
  // where the caller passed lmax <= 0 and some task turns that term on
  std::vector<double> lmr((size_t)ninst), lmc((size_t)ninst);
  for (int32_t k = 0; k < ninst; ++k) {
    lmr[(size_t)k] = inst[k].lmax_r_til;
    lmc[(size_t)k] = inst[k].lmax_c_til;
  }
  for (int32_t t = 0; t < ntasks; ++t) {
    const size_t k = (size_t)tasks[t].instance;
    if (tasks[t].gamma_r > 0 && !(lmr[k] > 0))
      STCHK(device_lmax(h, inst[k].Lr_til, kLmaxTol, kLmaxMaxIt, &lmr[k], nullptr, nullptr));
    if (tasks[t].gamma_c > 0 && !(lmc[k] > 0))
      STCHK(device_lmax(h, inst[k].Lc_til, kLmaxTol, kLmaxMaxIt, &lmc[k], nullptr, nullptr));
  }
  // ---- launch shape
  BatchCfg bc;
  bc.R = h->force_R > 0 ? h->force_R : 1;
  if (bc.R == 8) bc.R = 4;
  const size_t elem_cg = f32 ? sizeof(float) : sizeof(double);
  bc.lds = (size_t)bc.R * ld_max * sizeof(double) <= 65536;  // one shape serves FP64 and FP32
  if (h->force_lds == 0) bc.lds = false;
  BatchCfg fc;  // FISTA: sampled sizes, FP64
  fc.R = 1;
  fc.lds = (size_t)ldt_max * sizeof(double) <= 65536;

  // ---- task descriptors and workspace layout
  std::vector<BTask> bt((size_t)ntasks);
  std::vector<int> atab, ftab, vtab;
  Grids g;
  for (int32_t t = 0; t < ntasks; ++t) {
    const cpca_instance& I = inst[tasks[t].instance];
    const InstHost& H = ih[(size_t)tasks[t].instance];
    BTask& k = bt[(size_t)t];
    std::memset(&k, 0, sizeof k);
    k.p = (int)I.p;
    k.n = (int)I.n;
    k.ld = (int)H.ld;
    k.rho_r = (int)I.rho_r;
    k.rho_c = (int)I.rho_c;
    k.ldt = (int)H.ldt;
    k.gr = tasks[t].gamma_r;
    k.gc = tasks[t].gamma_c;
    const double beta = 2.0 * k.gc * lmc[(size_t)tasks[t].instance] +
                        2.0 * k.gr * lmr[(size_t)tasks[t].instance];
    k.lam = beta > 0.0 ? 1.0 / beta : 0.0;
    k.om_r = I.omega_r;
    k.om_c = I.omega_c;
    k.active = 1;
    k.inner_rel2 = 1e-10;
    k.floor2 = 0.0;
    k.keep_p = 0;
  }
  build_tables(bt, bc.R, atab, ftab, vtab, g);
  // the largest grids any candidate shape can need (R = 1)
  std::vector<BTask> bt1 = bt;
  std::vector<int> a1, f1, v1;
  Grids g1;
  build_tables(bt1, 1, a1, f1, v1, g1);

  char* img = nullptr;
  int *d_atab = nullptr, *d_ftab = nullptr, *d_vtab = nullptr;
  BTask* d_tasks = nullptr;
  CgScal* d_sc = nullptr;
  double *pa = nullptr, *pb = nullptr, *res = nullptr;
  std::vector<double*> Yi((size_t)ninst, nullptr);
  struct TaskBufs {
    double *S, *Za, *Zb, *B64, *X64, *r64, *p64, *q64;
    float *B32, *x32, *r32, *p32, *q32;
  };
  std::vector<TaskBufs> tb((size_t)ntasks);
  auto layout = [&](Arena& a) {
    img = a.take<char>(stg.buf.size());
    d_atab = a.take<int>(a1.size());
    d_ftab = a.take<int>(f1.size());
    d_vtab = a.take<int>(v1.size());
    d_tasks = a.take<BTask>((size_t)ntasks);
    d_sc = a.take<CgScal>((size_t)ntasks);
    pa = a.take<double>(2 * a1.size() + 16);
    pb = a.take<double>(2 * v1.size() + 16);
    res = a.take<double>((size_t)ntasks);
    for (int32_t k = 0; k < ninst; ++k)
      Yi[(size_t)k] = a.take<double>((size_t)inst[k].rho_r * ih[(size_t)k].ldt);
    for (int32_t t = 0; t < ntasks; ++t) {
      const BTask& k = bt[(size_t)t];
      TaskBufs& b = tb[(size_t)t];
      const size_t Nt = (size_t)k.rho_r * k.ldt, N = (size_t)k.p * k.ld;
      b = TaskBufs{};
      b.S = a.take<double>(Nt);
      b.Za = a.take<double>(Nt);
      b.Zb = a.take<double>(Nt);
      b.B64 = a.take<double>(N);
      b.X64 = a.take<double>(N);
      if (mode == CPCA_FP64) {
        b.r64 = a.take<double>(N);
        b.p64 = a.take<double>(N);
        b.q64 = a.take<double>(N);
      } else {
        if (mode == CPCA_FP32) b.B32 = a.take<float>(N);
        b.x32 = a.take<float>(N);
        b.r32 = a.take<float>(N);
        b.p32 = a.take<float>(N);
        b.q32 = a.take<float>(N);
      }
    }
  };
  {
    Arena a;
    layout(a);
    STCHK(ensure_ws(h, a.off));
  }
  Arena ar;
  ar.base = h->ws;
  layout(ar);
  HIPCHK(hipMemcpyAsync(img, stg.buf.data(), stg.buf.size(), hipMemcpyHostToDevice, h->stream));
  for (int32_t t = 0; t < ntasks; ++t) {
    BTask& k = bt[(size_t)t];
    const InstHost& H = ih[(size_t)tasks[t].instance];
    const DevGraph<double> d64 = bind_graph<double>(H.g64, img);
    const DevGraph<double> dt = bind_graph<double>(H.gt, img);
    k.Lr64 = d64.Lr;
    k.Lc64 = d64.Lc;
    k.mr = d64.mr;
    k.mc = d64.mc;
    if (f32) {
      const DevGraph<float> d32 = bind_graph<float>(H.g32, img);
      k.Lr32 = d32.Lr;
      k.Lc32 = d32.Lc;
    }
    k.Lrt = dt.Lr;
    k.Lct = dt.Lc;
    k.zmr = dt.mr;
    k.zmc = dt.mc;
    k.Y = Yi[(size_t)tasks[t].instance];
    const TaskBufs& b = tb[(size_t)t];
    k.S = b.S;
    k.Za = b.Za;
    k.Zb = b.Zb;
    k.B64 = b.B64;
    k.X64 = b.X64;
    k.r64 = b.r64;
    k.p64 = b.p64;
    k.q64 = b.q64;
    k.B32 = b.B32;
    k.x32 = b.x32;
    k.r32 = b.r32;
    k.p32 = b.p32;
    k.q32 = b.q32;
    k.sc = d_sc + t;
  }
  auto upload_tasks = [&]() -> cpca_status {
    HIPCHK(hipMemcpyAsync(d_tasks, bt.data(), sizeof(BTask) * bt.size(), hipMemcpyHostToDevice,
                          h->stream));
    HIPCHK(hipMemcpyAsync(d_atab, atab.data(), sizeof(int) * atab.size(), hipMemcpyHostToDevice,
                          h->stream));
    HIPCHK(hipMemcpyAsync(d_ftab, ftab.data(), sizeof(int) * ftab.size(), hipMemcpyHostToDevice,
                          h->stream));
    HIPCHK(hipMemcpyAsync(d_vtab, vtab.data(), sizeof(int) * vtab.size(), hipMemcpyHostToDevice,
                          h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));  // host vectors may change afterwards
    return CPCA_OK;
  };
  STCHK(upload_tasks());
  std::vector<CgScal> hsc((size_t)ntasks);
  auto read_sc = [&]() -> cpca_status {
    HIPCHK(hipMemcpyAsync(hsc.data(), d_sc, sizeof(CgScal) * hsc.size(), hipMemcpyDeviceToHost,
                          h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return prof_collect(h);
  };
  hipStream_t s = h->stream;

  // ---- FISTA for every task (FP64 state)
  for (int32_t k = 0; k < ninst; ++k) {
    const cpca_instance& I = inst[k];
    const size_t Nt = (size_t)I.rho_r * ih[(size_t)k].ldt;
    if (f32)
      k_copy_in<float><<<vec_grid(Nt), kThreads, 0, s>>>(Yi[(size_t)k], static_cast<const float*>(I.Ytil),
                                                         (int)I.rho_r, (int)I.rho_c, (int)ih[(size_t)k].ldt);
    else
      k_copy_in<double><<<vec_grid(Nt), kThreads, 0, s>>>(Yi[(size_t)k], static_cast<const double*>(I.Ytil),
                                                          (int)I.rho_r, (int)I.rho_c, (int)ih[(size_t)k].ldt);
    LAUNCHCHK();
  }
  k_fista_init_batched<<<g.v, kThreads, 0, s>>>(d_tasks, d_vtab);
  LAUNCHCHK();
  if (J > 0) {
    // capture the J FISTA launches once and replay them as one graph
    hipStream_t cs;
    HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipError_t err = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    double t = 1.0;
    for (int j = 1; j <= J && err == hipSuccess; ++j) {
      const double tn = (1.0 + std::sqrt(1.0 + 4.0 * t * t)) / 2.0;
      err = launch_bapply<double, B_FISTA>(h, cs, fc, g.f, (size_t)ldt_max, d_tasks, d_ftab,
                                           nullptr, (t - 1.0) / tn, (j - 1) & 1);
      t = tn;
    }
    hipError_t e2 = hipStreamEndCapture(cs, &graph);
    if (err == hipSuccess) err = e2;
    if (err == hipSuccess) err = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    hipEvent_t ev;
    if (err == hipSuccess) err = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (err == hipSuccess) {
      // order the graph after the set-up work on the handle stream
      err = hipEventRecord(ev, s);
      if (err == hipSuccess) err = hipStreamWaitEvent(cs, ev, 0);
      if (err == hipSuccess) err = hipGraphLaunch(exec, cs);
      if (err == hipSuccess) err = hipEventRecord(ev, cs);
      if (err == hipSuccess) err = hipStreamWaitEvent(s, ev, 0);
      const hipError_t e3 = hipStreamSynchronize(cs);
      if (err == hipSuccess) err = e3;
      (void)hipEventDestroy(ev);
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipStreamDestroy(cs);
    if (err != hipSuccess) return fail(CPCA_EHIP, std::string("batched FISTA: ") + hipGetErrorString(err));
  }
  for (int32_t t = 0; t < ntasks; ++t) {
    if (!tasks[t].Xtil_out) continue;
    const BTask& k = bt[(size_t)t];
    const size_t Nt = (size_t)k.rho_r * k.rho_c;
    if (f32)
      k_copy_out<float><<<vec_grid(Nt), kThreads, 0, s>>>(static_cast<float*>(tasks[t].Xtil_out), tb[(size_t)t].S,
                                                          k.rho_r, k.rho_c, k.ldt);
    else
      k_copy_out<double><<<vec_grid(Nt), kThreads, 0, s>>>(static_cast<double*>(tasks[t].Xtil_out), tb[(size_t)t].S,
                                                           k.rho_r, k.rho_c, k.ldt);
    LAUNCHCHK();
  }

  // ---- decoder right-hand sides: B = scatter(round(X~)), bb per task
  k_pass_batched<P_ZERO_B64><<<g.v, kThreads, 0, s>>>(d_tasks, d_vtab);
  LAUNCHCHK();
  if (f32)
    k_scatter_batched<float><<<g.v, kThreads, 0, s>>>(d_tasks, d_vtab);
  else
    k_scatter_batched<double><<<g.v, kThreads, 0, s>>>(d_tasks, d_vtab);
  LAUNCHCHK();
  k_bnorm_batched<<<ntasks, kThreads, 0, s>>>(d_tasks);
  LAUNCHCHK();
  STCHK(read_sc());
  std::vector<double> bb((size_t)ntasks);
  for (int32_t t = 0; t < ntasks; ++t) bb[(size_t)t] = hsc[(size_t)t].bb;

  // ---- autotune the batched CG product (or take the override)
  const bool cg32 = f32;
  auto cg_launch = [&](hipStream_t st, const BatchCfg& c, int grid, int par) -> hipError_t {
    return cg32 ? launch_bapply<float, B_CG32>(h, st, c, grid, (size_t)ld_max, d_tasks, d_atab, pa, 0.0, par)
                : launch_bapply<double, B_CG64>(h, st, c, grid, (size_t)ld_max, d_tasks, d_atab, pa, 0.0, par);
  };
  if (h->force_R == -1) {
    // candidates are timed on the right-hand sides (p = B after the first arm)
    int64_t sum_p = 0;
    for (const BTask& k : bt) sum_p += (int64_t)k.p * k.ld;
    const std::string key = tune_key(cg32 ? "batch32" : "batch64", elem_cg, ntasks, ld_max, sum_p);
    ApplyCfg best;
    if (!tune_lookup(h, key, best)) {
      // prepare p = B (rounded to the CG type) so that the candidates run
      // on meaningful data, and arm every task so none is skipped
      if (mode == CPCA_FP32_IR) {
        // FP32_IR keeps no FP32 copy of B: take the refinement residual at X = 0
        k_pass_batched<P_ZERO_X64><<<g.v, kThreads, 0, s>>>(d_tasks, d_vtab);
        LAUNCHCHK();
        k_pass_batched<P_ZERO_32><<<g.v, kThreads, 0, s>>>(d_tasks, d_vtab);
        LAUNCHCHK();
        HIPCHK((launch_bapply<double, B_RES>(h, s, bc, g.a, (size_t)ld_max, d_tasks, d_atab, pa,
                                             0.0, 0)));
        k_arm_batched<true><<<ntasks, kThreads, 0, s>>>(d_tasks, pa, 0.0);
        LAUNCHCHK();
      } else {
        if (mode == CPCA_FP32) k_pass_batched<P_B32><<<g.v, kThreads, 0, s>>>(d_tasks, d_vtab);
        if (cg32) k_init_zero_batched<float><<<g.v, kThreads, 0, s>>>(d_tasks, d_vtab, pb);
        else k_init_zero_batched<double><<<g.v, kThreads, 0, s>>>(d_tasks, d_vtab, pb);
        LAUNCHCHK();
        k_arm_batched<false><<<ntasks, kThreads, 0, s>>>(d_tasks, pb, 1e-300);
        LAUNCHCHK();
      }
      ApplyCfg base;
      base.vec = (int)(16 / elem_cg);
      STCHK(autotune(h, key, ld_max, sizeof(double), base,
                     [&](const ApplyCfg& c) -> cpca_status {
                       BatchCfg b2{c.R, c.lds};
                       std::vector<BTask> btc = bt;
                       std::vector<int> at, ft, vt;
                       Grids gc2;
                       build_tables(btc, c.R, at, ft, vt, gc2);
                       HIPCHK(hipMemcpyAsync(d_tasks, btc.data(), sizeof(BTask) * btc.size(),
                                             hipMemcpyHostToDevice, s));
                       HIPCHK(hipMemcpyAsync(d_atab, at.data(), sizeof(int) * at.size(),
                                             hipMemcpyHostToDevice, s));
                       HIPCHK(hipStreamSynchronize(s));
                       const hipError_t e = cg_launch(s, b2, gc2.a, 0);
                       if (e != hipSuccess) return fail(CPCA_EHIP, hipGetErrorString(e));
                       return CPCA_OK;
                     },
                     &best));
    }
    bc.R = best.R;
    bc.lds = best.lds;
    build_tables(bt, bc.R, atab, ftab, vtab, g);
    STCHK(upload_tasks());
  }

  // ---- CG over all tasks, chunks of iterations replayed as a graph
  constexpr int kChunk = 16;  // even: the parity of every replay matches the capture
  // Tail compaction: once at most half of the tasks in the current block
  // tables are still running, the tables are rebuilt over the running tasks
  // and the chunk graph is captured again, so that the slow tasks at the end
  // no longer launch a workgroup per row block of every converged task. A
  // task keeps its own block order and reduction order, so results are
  // unchanged. The full tables are restored before returning.
  auto run_cg = [&](int max_it, int* ran) -> cpca_status {
    hipStream_t cs;
    HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipEvent_t ev;
    HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    Grids gr = g;  // grids of the tables on the device
    auto enqueue_iter = [&](hipStream_t st, int par) -> hipError_t {
      hipError_t e = cg_launch(st, bc, gr.a, par);
      if (e != hipSuccess) return e;
      if (cg32) {
        k_update_batched<float><<<gr.v, kThreads, 0, st>>>(d_tasks, d_vtab, pa, pb, par);
        k_pupdate_batched<float><<<gr.v, kThreads, 0, st>>>(d_tasks, d_vtab, pb, par);
      } else {
        k_update_batched<double><<<gr.v, kThreads, 0, st>>>(d_tasks, d_vtab, pa, pb, par);
        k_pupdate_batched<double><<<gr.v, kThreads, 0, st>>>(d_tasks, d_vtab, pb, par);
      }
      return hipGetLastError();
    };
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    auto capture = [&]() -> hipError_t {
      if (exec) (void)hipGraphExecDestroy(exec);
      if (graph) (void)hipGraphDestroy(graph);
      exec = nullptr;
      graph = nullptr;
      if (max_it < kChunk) return hipSuccess;
      hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
      for (int k = 0; k < kChunk && e == hipSuccess; ++k) e = enqueue_iter(cs, k & 1);
      const hipError_t e2 = hipStreamEndCapture(cs, &graph);
      if (e == hipSuccess) e = e2;
      if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      return e;
    };
    // the tables of the running tasks; called with the streams idle
    int in_tables = ntasks;
    bool compacted = false;
    std::vector<char> live((size_t)ntasks, 0);
    std::vector<BTask> btc;
    std::vector<int> atc, ftc, vtc;
    auto compact = [&](int n_live, int it_now) -> hipError_t {
      btc = bt;
      build_tables(btc, bc.R, atc, ftc, vtc, gr, &live);
      hipError_t e = hipMemcpyAsync(d_tasks, btc.data(), sizeof(BTask) * btc.size(),
                                    hipMemcpyHostToDevice, s);
      if (e == hipSuccess)
        e = hipMemcpyAsync(d_atab, atc.data(), sizeof(int) * atc.size(), hipMemcpyHostToDevice, s);
      if (e == hipSuccess)
        e = hipMemcpyAsync(d_vtab, vtc.data(), sizeof(int) * vtc.size(), hipMemcpyHostToDevice, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (h->debug)
        std::fprintf(stderr, "[cpca] batched CG: tables compacted from %d to %d tasks at iteration %d\n",
                     in_tables, n_live, it_now);
      in_tables = n_live;
      compacted = true;
      return e;
    };
    hipError_t err = hipSuccess;
    if (h->batch_compact) {
      int n_live = 0;
      for (int32_t t = 0; t < ntasks; ++t) {
        live[(size_t)t] = bt[(size_t)t].active ? 1 : 0;
        n_live += live[(size_t)t];
      }
      if (n_live > 0 && 2 * n_live <= in_tables) err = compact(n_live, 0);
    }
    if (err == hipSuccess) err = capture();
    int it = 0;
    cpca_status st = CPCA_OK;
    if (err == hipSuccess) err = hipEventRecord(ev, s);
    if (err == hipSuccess) err = hipStreamWaitEvent(cs, ev, 0);
    while (err == hipSuccess && it < max_it) {
      if (exec && it + kChunk <= max_it) {
        err = hipGraphLaunch(exec, cs);
        it += kChunk;
      } else {
        err = enqueue_iter(cs, it & 1);
        it += 1;
      }
      if (err == hipSuccess) err = hipEventRecord(ev, cs);
      if (err == hipSuccess) err = hipStreamWaitEvent(s, ev, 0);
      if (err != hipSuccess) break;
      if ((st = read_sc()) != CPCA_OK) break;  // both streams are idle after this
      int n_live = 0;
      for (int32_t t = 0; t < ntasks; ++t) {
        live[(size_t)t] = hsc[(size_t)t].done == 0 ? 1 : 0;
        n_live += live[(size_t)t];
      }
      if (n_live == 0) break;
      // recapture only while whole chunks remain (the parity of the next
      // iteration is even there, as in the capture)
      if (h->batch_compact && exec && 2 * n_live <= in_tables && it + kChunk <= max_it) {
        err = compact(n_live, it);
        if (err == hipSuccess) err = capture();
      }
    }
    const hipError_t e3 = hipStreamSynchronize(cs);
    if (err == hipSuccess) err = e3;
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipEventDestroy(ev);
    (void)hipStreamDestroy(cs);
    if (err != hipSuccess) return fail(CPCA_EHIP, std::string("batched CG: ") + hipGetErrorString(err));
    if (compacted) STCHK(upload_tasks());
    *ran = it;
    return st;
  };

  std::vector<int> iters((size_t)ntasks, 0), outer((size_t)ntasks, 0), done((size_t)ntasks, 0);
  const double tol2 = tol * tol;
  if (mode != CPCA_FP32_IR) {
    if (mode == CPCA_FP32) k_pass_batched<P_B32><<<g.v, kThreads, 0, s>>>(d_tasks, d_vtab);
    if (cg32) k_init_zero_batched<float><<<g.v, kThreads, 0, s>>>(d_tasks, d_vtab, pb);
    else k_init_zero_batched<double><<<g.v, kThreads, 0, s>>>(d_tasks, d_vtab, pb);
    LAUNCHCHK();
    k_arm_batched<false><<<ntasks, kThreads, 0, s>>>(d_tasks, pb, tol2);
    LAUNCHCHK();
    int ran = 0;
    STCHK(run_cg(max_iter, &ran));
    STCHK(read_sc());
    for (int32_t t = 0; t < ntasks; ++t) {
      iters[(size_t)t] = hsc[(size_t)t].iter;
      done[(size_t)t] = hsc[(size_t)t].done;
    }
    if (mode == CPCA_FP32) {
      k_pass_batched<P_X64_FROM_32><<<g.v, kThreads, 0, s>>>(d_tasks, d_vtab);
      LAUNCHCHK();
    }
  } else {
    k_pass_batched<P_ZERO_X64><<<g.v, kThreads, 0, s>>>(d_tasks, d_vtab);
    LAUNCHCHK();
    k_pass_batched<P_ZERO_32><<<g.v, kThreads, 0, s>>>(d_tasks, d_vtab);
    LAUNCHCHK();
    // FP32 CG with FP64 residual replacement (as in the single-problem
    // solver): each segment runs until its recursive residual has dropped by
    // kReplace against the last true residual (or to (0.3 tol)^2 ||B||^2);
    // then X64 += x32 and the true residual replaces the FP32 one, keeping
    // the direction. A task whose segment fails (breakdown, NaN/Inf,
    // divergence: X64 is left untouched), does not lower the true residual,
    // or needs more than kSlow times the iterations per decade of true-
    // residual reduction of its first segment is too ill-conditioned for the
    // FP32 recursion to carry a direction across replacements; it switches to
    // restarted refinement (p = r at every segment, inner tolerance
    // clamp(0.5 tol / rel, 1e-5, 0.25)). kMaxBad failed segments in a row end
    // the task.
    constexpr double kReplace2 = 1e-4;
    constexpr int kMaxBad = 3;
    std::vector<int> bad_run((size_t)ntasks, 0), last_bad((size_t)ntasks, 0);
    std::vector<double> rel_prev((size_t)ntasks, HUGE_VAL);
    std::vector<char> keep((size_t)ntasks, 0);     // the first residual pass sets p = r
    std::vector<char> restart((size_t)ntasks, h->ir_restart ? 1 : 0);  // restarted refinement
    constexpr double kSlow = 2.2;
    std::vector<double> ipd_first((size_t)ntasks, 0.0);
    std::vector<int> seg_iters((size_t)ntasks, 0);
    for (int o = 0;; ++o) {
      bool any = false;
      for (int32_t t = 0; t < ntasks; ++t) {
        BTask& k = bt[(size_t)t];
        if (restart[(size_t)t]) {
          const double it_tol =
              std::min(0.25, std::max(1e-5, 0.5 * tol / std::min(1.0, rel_prev[(size_t)t])));
          k.inner_rel2 = it_tol * it_tol;
          k.floor2 = 0.0;
          k.keep_p = 0;
        } else {
          k.inner_rel2 = kReplace2;
          k.floor2 = 0.09 * tol2 * bb[(size_t)t];
          k.keep_p = keep[(size_t)t];
        }
        k.reset_p = 0;
        any = any || k.active;
      }
      if (!any) break;
      STCHK(upload_tasks());
      HIPCHK((launch_bapply<double, B_RES>(h, s, bc, g.a, (size_t)ld_max, d_tasks, d_atab, pa, 0.0, 0)));
      k_arm_batched<true><<<ntasks, kThreads, 0, s>>>(d_tasks, pa, 0.0);
      LAUNCHCHK();
      STCHK(read_sc());
      bool need = false, reset = false;
      for (int32_t t = 0; t < ntasks; ++t) {
        BTask& k = bt[(size_t)t];
        if (!k.active) continue;
        const CgScal& c = hsc[(size_t)t];
        const double rel = bb[(size_t)t] > 0 ? std::sqrt(c.res2 / bb[(size_t)t]) : 0.0;
        outer[(size_t)t] = o;
        if (c.done == 3 || !std::isfinite(c.res2)) {
          done[(size_t)t] = 3;
          k.active = 0;
        } else if (rel <= tol) {
          done[(size_t)t] = 1;
          k.active = 0;
        } else if (bad_run[(size_t)t] >= kMaxBad) {
          done[(size_t)t] = last_bad[(size_t)t];
          k.active = 0;
        } else if (o >= kMaxOuter) {
          done[(size_t)t] = 0;
          k.active = 0;
        } else {
          bool slow = false;
          if (o > 0 && rel < rel_prev[(size_t)t] && seg_iters[(size_t)t] > 0) {
            const double ipd = seg_iters[(size_t)t] / std::log10(rel_prev[(size_t)t] / rel);
            if (ipd_first[(size_t)t] == 0.0) ipd_first[(size_t)t] = ipd;
            else slow = ipd > kSlow * ipd_first[(size_t)t];
          }
          if (k.keep_p && (!(rel < rel_prev[(size_t)t]) || slow)) {  // no or slowing progress
            k.reset_p = 1;
            reset = true;
            restart[(size_t)t] = 1;
            const double it_tol = std::min(0.25, std::max(1e-5, 0.5 * tol / std::min(1.0, rel)));
            k.inner_rel2 = it_tol * it_tol;
            k.floor2 = 0.0;
          }
          rel_prev[(size_t)t] = rel;
          need = true;
        }
      }
      if (!need) break;
      STCHK(upload_tasks());
      if (reset) {
        k_pass_batched<P_P_FROM_R><<<g.v, kThreads, 0, s>>>(d_tasks, d_vtab);
        LAUNCHCHK();
      }
      // re-arm from the same residual partials so that the tasks found
      // converged above are marked done before the inner solves
      k_arm_batched<true><<<ntasks, kThreads, 0, s>>>(d_tasks, pa, 0.0);
      LAUNCHCHK();
      int ran = 0;
      STCHK(run_cg(max_iter, &ran));
      STCHK(read_sc());
      for (int32_t t = 0; t < ntasks; ++t) {
        BTask& k = bt[(size_t)t];
        if (!k.active) continue;
        const CgScal& c = hsc[(size_t)t];
        iters[(size_t)t] += c.iter;
        seg_iters[(size_t)t] = c.iter;
        const bool failed = c.done == 2 || c.done == 3 || c.done == 4;
        bad_run[(size_t)t] = failed ? bad_run[(size_t)t] + 1 : 0;
        if (failed) {
          last_bad[(size_t)t] = c.done == 4 ? 0 : c.done;
          restart[(size_t)t] = 1;
        }
        keep[(size_t)t] = !failed && c.done == 1;
      }
      // X64 += x32 for the tasks whose segment did not fail (the pass checks)
      k_pass_batched<P_ACCUM><<<g.v, kThreads, 0, s>>>(d_tasks, d_vtab);
      LAUNCHCHK();
    }
  }

  // ---- FP64 residual per task, outputs
  HIPCHK((launch_bapply<double, B_RESNORM>(h, s, bc, g.a, (size_t)ld_max, d_tasks, d_atab, pa, 0.0, 0)));
  k_apply_sum_batched<1><<<ntasks, kThreads, 0, s>>>(d_tasks, pa, res);
  LAUNCHCHK();
  for (int32_t t = 0; t < ntasks; ++t) {
    const BTask& k = bt[(size_t)t];
    const size_t N = (size_t)k.p * k.n;
    if (f32)
      k_copy_out<float><<<vec_grid(N), kThreads, 0, s>>>(static_cast<float*>(tasks[t].X_out), tb[(size_t)t].X64,
                                                         k.p, k.n, k.ld);
    else
      k_copy_out<double><<<vec_grid(N), kThreads, 0, s>>>(static_cast<double*>(tasks[t].X_out), tb[(size_t)t].X64,
                                                          k.p, k.n, k.ld);
    LAUNCHCHK();
  }
  std::vector<double> hres((size_t)ntasks);
  HIPCHK(hipMemcpyAsync(hres.data(), res, sizeof(double) * ntasks, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  STCHK(prof_collect(h));
  cpca_status worst = CPCA_OK;
  for (int32_t t = 0; t < ntasks; ++t) {
    const double rel = bb[(size_t)t] > 0 ? std::sqrt(hres[(size_t)t] / bb[(size_t)t]) : 0.0;
    cpca_status st = CPCA_OK;
    switch (done[(size_t)t]) {
      case 1: st = CPCA_OK; break;
      case 2: st = CPCA_ENOTSPD; break;
      case 3: st = CPCA_ENAN; break;
      default: st = CPCA_ENOCONV; break;
    }
    if (bb[(size_t)t] == 0.0) st = CPCA_OK;
    if (st != CPCA_OK && (worst == CPCA_OK || worst == CPCA_ENOCONV)) worst = st;
    if (infos) fill_info(&infos[t], st, iters[(size_t)t], outer[(size_t)t], rel, 0.0, t0);
  }
  if (worst != CPCA_OK) {
    char buf[96];
    std::snprintf(buf, sizeof buf, "batched: at least one task ended with status %d", (int)worst);
    return fail(worst, buf);
  }
  return CPCA_OK;
}

}  // namespace

extern "C" cpca_status cpca_solve_batched(cpca_handle h, cpca_mode mode,
                                          const cpca_instance* instances, int32_t n_instances,
                                          const cpca_task* tasks, int32_t n_tasks,
                                          int32_t fista_iters, double tol, int32_t max_iter,
                                          cpca_info* infos) {
  TraceRange trace_("cpca_solve_batched");
  clear_error();
  STCHK(check_batched_args(mode, instances, n_instances, tasks, n_tasks, fista_iters, tol,
                           max_iter));
  if (!h) return fail(CPCA_EINVAL, "null handle");
  return run_batched(h, mode, instances, n_instances, tasks, n_tasks, fista_iters, tol, max_iter,
                     infos);
}
