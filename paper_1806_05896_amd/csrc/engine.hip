// Serving engine: continuous batching of IPM solves.
//
// Requests (a problem plus its options) wait in a FIFO queue and are
// admitted while a slot is free and the sum of the admitted problems' HBM
// footprints stays within the budget; admission allocates a problem's
// Newton/Krylov/multigrid workspace and retirement frees it, while the
// problem data and iterates stay on the device for the caller to query.
// Every engine step advances each admitted request by one iteration of
// Algorithm A.1 (Appendix): requests that share the Krylov and multigrid
// options form one group, whose kernels advance all its members in the same
// launches.  A request that arrives while others run joins at the next
// step, starting from its own initial point, so requests at different IPM
// iterations share every launch.  Each request takes exactly the arithmetic
// of a solo solve (per-instance reductions and kernel choices), so its
// result does not depend on what else is in flight.  The groups of one step
// run concurrently, each on a stream of its own driven by a host thread of
// its own, so the latency-bound launches of one overlap those of another.

using Clock = std::chrono::steady_clock;

struct EngineReq {
  uint64_t ticket = 0;
  ipmpde_problem* P = nullptr;
  ipmpde_options o;
  size_t bytes = 0;
  Clock::time_point t_submit, t_admit, t_done;
  int state = IPMPDE_REQ_QUEUED;
  int k = 0;           // IPM iteration whose measures come next
  bool fresh = true;   // still to be put at the starting point
};

struct EngineClass {
  ipmpde_options o;  // Krylov and multigrid options of every member
  int dim = 0;
  bool q1 = false;   // Q1 problems (a group holds them or none)
  int band = 0;      // size band of the members (engine_band)
  Group* G = nullptr;
  hipStream_t stream = nullptr;  // the class's stream (default priority), also its group's capture stream
  hipEvent_t done = nullptr;     // the class's stream at the end of a step
  bool any_fresh = false;        // a member still to be put at its starting point
  std::vector<EngineReq*> members;
};

static void engine_class_free(EngineClass* C) {
  group_release(C->G);
  if (C->stream) (void)hipStreamDestroy(C->stream);
  if (C->done) (void)hipEventDestroy(C->done);
  delete C;
}

struct ipmpde_engine {
  size_t budget = 0, in_use = 0, peak = 0;
  int max_slots = 0, running = 0;
  uint64_t next_ticket = 1;
  long steps = 0;
  std::deque<EngineReq*> queue;
  std::vector<EngineClass*> classes;
  std::map<uint64_t, EngineReq*> reqs;
  hipEvent_t start_ev = nullptr;  // the caller's stream at the start of a step
};

static bool same_solver(const ipmpde_options& a, const ipmpde_options& b) {
  return a.krylov == b.krylov && a.precond == b.precond && a.restart == b.restart && a.krylov_tol == b.krylov_tol &&
         a.krylov_maxit == b.krylov_maxit && a.nu_pre == b.nu_pre && a.nu_post == b.nu_post && a.omega == b.omega &&
         a.mg_precision == b.mg_precision && a.chunk == b.chunk && a.use_graphs == b.use_graphs &&
         a.vcycles == b.vcycles && a.mg_tile == b.mg_tile;
}

// Requests are grouped by size as well as by solver options: a group's
// launches cover its largest member and each Krylov chunk runs until its
// slowest member stops, so small requests beside large ones would wait on
// them, while groups of different bands run concurrently.
static int engine_band(const ipmpde_problem* P) { return P->n > 8192 ? 1 : 0; }

static int next_pow2(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

extern "C" int ipmpde_engine_create(size_t hbm_budget_bytes, int max_slots, ipmpde_engine** out) {
  if (!out) return fail(IPMPDE_EINVAL, "out is NULL");
  *out = nullptr;
  if (hbm_budget_bytes == 0) return fail(IPMPDE_EINVAL, "hbm_budget_bytes must be positive");
  if (max_slots < 1 || max_slots > 4096) return fail(IPMPDE_EINVAL, "max_slots must be in [1, 4096]");
  ipmpde_engine* E = new ipmpde_engine();
  E->budget = hbm_budget_bytes;
  E->max_slots = max_slots;
  *out = E;
  return IPMPDE_OK;
}

static void engine_retire(ipmpde_engine* E, EngineReq* R, int status) {
  R->P->stats.status = status;
  R->t_done = Clock::now();
  R->P->stats.solve_ms = std::chrono::duration<double, std::milli>(R->t_done - R->t_admit).count();
  R->state = IPMPDE_REQ_DONE;
  release_work(R->P);
  R->P->in_engine = false;
  E->in_use -= R->bytes;
  E->running -= 1;
}

extern "C" void ipmpde_engine_destroy(ipmpde_engine* E) {
  if (!E) return;
  (void)hipDeviceSynchronize();
  for (auto& kv : E->reqs) {
    EngineReq* R = kv.second;
    if (R->state == IPMPDE_REQ_RUNNING) release_work(R->P);
    if (R->state != IPMPDE_REQ_DONE) R->P->in_engine = false;
    delete R;
  }
  for (EngineClass* C : E->classes) engine_class_free(C);
  if (E->start_ev) (void)hipEventDestroy(E->start_ev);
  delete E;
}

extern "C" int ipmpde_engine_submit(ipmpde_engine* E, ipmpde_problem* P, const ipmpde_options* opts,
                                    uint64_t* ticket) {
  if (!E || !P || !ticket) return fail(IPMPDE_EINVAL, "NULL argument");
  if (P->in_engine) return fail(IPMPDE_EINVAL, "problem is already queued or running in an engine");
  if (P->pde == IPMPDE_HEAT) return fail(IPMPDE_EINVAL, "heat-equation problems are not served by the engine");
  ipmpde_options o;
  TRY(resolve_opts(opts, &o));
  if (o.mass_scaling != IPMPDE_MASS_UNIT) return fail(IPMPDE_EINVAL, "the engine serves the unit-mass form only");
  P->rep = 1.0;
  ipmpde_grid g{P->dim, P->N};
  ipmpde_pde d{P->pde, P->eps};
  const size_t bytes = ipmpde_footprint_bytes(&g, &d, P->has_y ? 1 : 0, &o);
  if (bytes > E->budget) return fail(IPMPDE_ENOMEM, "the request's footprint exceeds the engine's HBM budget");
  EngineReq* R = new EngineReq();
  R->ticket = E->next_ticket++;
  R->P = P;
  R->o = o;
  R->bytes = bytes;
  R->t_submit = Clock::now();
  P->in_engine = true;
  E->queue.push_back(R);
  E->reqs[R->ticket] = R;
  *ticket = R->ticket;
  return IPMPDE_OK;
}

// Move queued requests into free slots, in arrival order, while the budget
// allows (the head of the queue is never overtaken).
static int engine_admit(ipmpde_engine* E) {
  while (!E->queue.empty() && E->running < E->max_slots) {
    EngineReq* R = E->queue.front();
    if (E->in_use + R->bytes > E->budget) break;
    E->queue.pop_front();
    EngineClass* C = nullptr;
    const bool q1 = R->P->pde == IPMPDE_POISSON_Q1;
    const int band = engine_band(R->P);
    for (EngineClass* c : E->classes)
      if (c->dim == R->P->dim && c->q1 == q1 && c->band == band && same_solver(c->o, R->o)) C = c;
    if (!C) {
      C = new EngineClass();
      C->o = R->o;
      C->dim = R->P->dim;
      C->q1 = q1;
      C->band = band;
      int rc = group_create({}, E->max_slots, C->dim, &C->G);
      hipError_t e = hipSuccess;
      if (rc == IPMPDE_OK && (e = hipStreamCreateWithFlags(&C->stream, hipStreamNonBlocking)) == hipSuccess)
        e = hipEventCreateWithFlags(&C->done, hipEventDisableTiming);
      if (rc == IPMPDE_OK && e != hipSuccess)
        rc = fail(IPMPDE_EDEVICE, std::string("engine class setup: ") + hipGetErrorString(e));
      if (rc != IPMPDE_OK) {
        engine_class_free(C);
        E->queue.push_front(R);
        return rc;
      }
      C->G->q1 = q1;
      C->G->cap_stream = C->stream;
      C->G->own_cap = false;
      E->classes.push_back(C);
    }
    R->t_admit = Clock::now();
    R->state = IPMPDE_REQ_RUNNING;
    R->fresh = true;
    R->k = 0;
    ipm_begin(R->P);
    E->in_use += R->bytes;
    E->peak = std::max(E->peak, E->in_use);
    E->running += 1;
    const int rc = ensure_work(R->P);
    if (rc != IPMPDE_OK) {
      engine_retire(E, R, rc);
      continue;
    }
    C->members.push_back(R);
  }
  return IPMPDE_OK;
}

// The members and descriptors of one class for this step; runs on the
// calling thread (group_select allocates the multigrid levels a member has
// not used yet).
static int engine_class_prepare(EngineClass* C) {
  Group* G = C->G;
  const int m = (int)C->members.size();
  G->probs.resize(m);
  G->count = m;
  G->zc = std::min(next_pow2(m), G->cap);
  C->any_fresh = false;
  for (int i = 0; i < m; ++i) {
    EngineReq* R = C->members[i];
    G->probs[i] = R->P;
    G->H[i].active = 1;
    G->H[i].mu = R->P->mu;
    G->H[i].alpha0 = R->o.alpha0;
    C->any_fresh = C->any_fresh || R->fresh;
  }
  return group_select(G, C->o);
}

// One IPM iteration of every member of one class on stream s; fin[i] >= 0
// is the final status of a member that has finished.  Touches only the
// class, its group and its members' problems.
static int engine_class_run(EngineClass* C, hipStream_t s, std::vector<int>& fin) {
  Group* G = C->G;
  const int m = (int)C->members.size();
  if (C->any_fresh) {
    // the starting point of the new members only
    for (int i = 0; i < m; ++i) {
      EngineReq* R = C->members[i];
      G->H[i].active = R->fresh ? 1 : 0;
      if (R->fresh) {
        R->P->mu = R->o.mu0;
        G->H[i].mu = R->o.mu0;
      }
    }
    TRY(group_sync(G, s));
    hipLaunchKernelGGL(k_init_state, gz(G, G->max_n), dim3(kBS), 0, s, G->D);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));  // the upload above has read the flags
    for (int i = 0; i < m; ++i) {
      C->members[i]->fresh = false;
      C->members[i]->P->need_init = false;
      G->H[i].active = 1;
    }
  }
  bool mean = false;
  for (const EngineReq* R : C->members) mean = mean || R->o.mu_rule == IPMPDE_MU_CENTRAL;
  TRY(group_measures(G, s, mean));
  fin.assign(m, -1);
  int alive = 0;
  for (int i = 0; i < m; ++i) {
    fin[i] = ipm_check(G, i, C->members[i]->k, C->members[i]->o);
    if (fin[i] < 0) ++alive;
  }
  if (alive) {
    TRY(group_step(G, C->o, s));
    for (int i = 0; i < m; ++i) {
      if (fin[i] >= 0) continue;
      fin[i] = ipm_after_step(G, i, C->members[i]->k);
      C->members[i]->k += 1;
    }
  }
  return IPMPDE_OK;
}

// Retire the finished members (calling thread).  The class's stream is idle
// here (group_step and group_measures end with a read-back), so their
// workspace can go.
static void engine_class_finish(ipmpde_engine* E, EngineClass* C, const std::vector<int>& fin) {
  std::vector<EngineReq*> keep;
  for (size_t i = 0; i < C->members.size(); ++i) {
    if (i < fin.size() && fin[i] >= 0) engine_retire(E, C->members[i], fin[i]);
    else keep.push_back(C->members[i]);
  }
  C->members.swap(keep);
}

extern "C" int ipmpde_engine_step(ipmpde_engine* E, ipmpde_stream stream, int* running, int* queued) {
  if (!E) return fail(IPMPDE_EINVAL, "engine is NULL");
  hipStream_t s = S(stream);
  TRY(engine_admit(E));
  std::vector<EngineClass*> act;
  for (EngineClass* C : E->classes)
    if (!C->members.empty()) act.push_back(C);
  for (EngineClass* C : act) TRY(engine_class_prepare(C));
  if (!act.empty()) {
    if (!E->start_ev) HIP_TRY(hipEventCreateWithFlags(&E->start_ev, hipEventDisableTiming));
    HIP_TRY(hipEventRecord(E->start_ev, s));
    for (EngineClass* C : act) HIP_TRY(hipStreamWaitEvent(C->stream, E->start_ev, 0));
    const size_t na = act.size();
    std::vector<std::vector<int>> fin(na);
    std::vector<int> rc(na, IPMPDE_OK);
    std::vector<std::string> msg(na);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    auto run = [&](size_t k) {
      if (k > 0) {
        const hipError_t e = hipSetDevice(dev);
        if (e != hipSuccess) {
          rc[k] = IPMPDE_EDEVICE;
          msg[k] = std::string("hipSetDevice: ") + hipGetErrorString(e);
          return;
        }
      }
      rc[k] = engine_class_run(act[k], act[k]->stream, fin[k]);
      if (rc[k] != IPMPDE_OK) msg[k] = g_err;
    };
    std::vector<std::thread> th;
    try {
      for (size_t k = 1; k < na; ++k) th.emplace_back(run, k);
    } catch (const std::exception& ex) {
      for (size_t k = th.size() + 1; k < na; ++k) {
        rc[k] = IPMPDE_EDEVICE;
        msg[k] = std::string("cannot start a class thread: ") + ex.what();
      }
    }
    run(0);
    for (auto& t : th) t.join();
    for (EngineClass* C : act) {
      HIP_TRY(hipEventRecord(C->done, C->stream));
      HIP_TRY(hipStreamWaitEvent(s, C->done, 0));
    }
    int first = -1;
    for (size_t k = 0; k < na; ++k) {
      if (rc[k] == IPMPDE_OK) engine_class_finish(E, act[k], fin[k]);
      else if (first < 0) first = (int)k;
    }
    if (first >= 0) return fail(rc[first], msg[first]);
  }
  E->steps += 1;
  if (running) *running = E->running;
  if (queued) *queued = (int)E->queue.size();
  return IPMPDE_OK;
}

extern "C" int ipmpde_engine_poll(const ipmpde_engine* E, uint64_t ticket, ipmpde_request_info* info) {
  if (!E || !info) return fail(IPMPDE_EINVAL, "NULL argument");
  auto it = E->reqs.find(ticket);
  if (it == E->reqs.end()) return fail(IPMPDE_EINVAL, "unknown ticket");
  const EngineReq* R = it->second;
  const auto ms = [](Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
  };
  const Clock::time_point now = Clock::now();
  std::memset(info, 0, sizeof(*info));
  info->state = R->state;
  info->status = R->state == IPMPDE_REQ_DONE ? R->P->stats.status : -1;
  info->nli = R->state == IPMPDE_REQ_QUEUED ? 0 : R->P->stats.nli;
  info->krylov_its = R->state == IPMPDE_REQ_QUEUED ? 0 : R->P->stats.krylov_its;
  info->queue_ms = ms(R->t_submit, R->state == IPMPDE_REQ_QUEUED ? now : R->t_admit);
  info->latency_ms = ms(R->t_submit, R->state == IPMPDE_REQ_DONE ? R->t_done : now);
  info->footprint_bytes = R->bytes;
  return IPMPDE_OK;
}

extern "C" int ipmpde_engine_release(ipmpde_engine* E, uint64_t ticket) {
  if (!E) return fail(IPMPDE_EINVAL, "engine is NULL");
  auto it = E->reqs.find(ticket);
  if (it == E->reqs.end()) return fail(IPMPDE_EINVAL, "unknown ticket");
  if (it->second->state != IPMPDE_REQ_DONE) return fail(IPMPDE_EINVAL, "request has not finished");
  delete it->second;
  E->reqs.erase(it);
  return IPMPDE_OK;
}

extern "C" int ipmpde_engine_get_info(const ipmpde_engine* E, ipmpde_engine_info* info) {
  if (!E || !info) return fail(IPMPDE_EINVAL, "NULL argument");
  std::memset(info, 0, sizeof(*info));
  info->running = E->running;
  info->queued = (int)E->queue.size();
  info->groups = 0;
  for (const EngineClass* C : E->classes) info->groups += C->members.empty() ? 0 : 1;
  info->bytes_in_use = E->in_use;
  info->peak_bytes = E->peak;
  info->budget_bytes = E->budget;
  info->steps = E->steps;
  return IPMPDE_OK;
}
