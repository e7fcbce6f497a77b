// Autotuner of a batch's multigrid schedule: V-cycles per solve, Jacobi
// sweeps, the tile size of the 2D Poisson level kernels, (optionally) the
// V-cycle precision, and the number of lanes the instances are split into,
// picked by timing whole batched solves.  Results are kept
// in a JSON file keyed by the GPU architecture and the batch's shape, so a
// shape is tuned once per machine type.

namespace {

struct TuneEntry {
  int vcycles = 1, nu_pre = 2, nu_post = 2, mg_precision = IPMPDE_FP32, mg_tile = IPMPDE_TILE_AUTO, lanes = 1;
  double ms = 0;
};

std::string device_arch() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  std::string a = prop.gcnArchName;
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

// Hardware queues HIP gives the process (GPU_MAX_HW_QUEUES, 4 when unset):
// lanes whose streams share a queue run one after the other, so the best lane
// count depends on it.
int hw_queues() {
  const char* v = std::getenv("GPU_MAX_HW_QUEUES");
  const int q = v ? std::atoi(v) : 0;
  return q > 0 ? q : 4;
}

// arch/d<dim>/pde<mask of kinds>/N<largest N>/nt<largest nt>/x<count>/kry<k>/pc<p>/y<state bounds>/r<restart>/
// mp<precision or -1 when tuned>/q<hardware queues>
std::string tune_key(const Group* G, const ipmpde_options& o, int flags) {
  int maxN = 0, maxnt = 1, mask = 0, any_y = 0;
  for (const ipmpde_problem* P : G->probs) {
    maxN = std::max(maxN, P->N);
    maxnt = std::max(maxnt, P->nt);
    mask |= 1 << P->pde;
    any_y |= P->has_y ? 1 : 0;
  }
  char buf[256];
  std::snprintf(buf, sizeof buf, "%s/d%d/pde%d/N%d/nt%d/x%d/kry%d/pc%d/y%d/r%d/mp%d/q%d", device_arch().c_str(),
                G->dim, mask, maxN, maxnt, G->count, o.krylov, o.precond, any_y,
                o.krylov == IPMPDE_FGMRES ? o.restart : 0, (flags & IPMPDE_TUNE_PRECISION) ? -1 : o.mg_precision,
                hw_queues());
  return buf;
}

// The cache: one entry per line, `  "key": {"vcycles": v, ...}` inside a
// JSON object (entries written before lanes were tuned read as one lane).
std::map<std::string, TuneEntry> read_cache(const char* path) {
  std::map<std::string, TuneEntry> m;
  FILE* f = std::fopen(path, "r");
  if (!f) return m;
  char line[1024];
  while (std::fgets(line, sizeof line, f)) {
    const char* q0 = std::strchr(line, '"');
    if (!q0) continue;
    const char* q1 = std::strchr(q0 + 1, '"');
    if (!q1) continue;
    TuneEntry e;
    if (std::sscanf(q1 + 1,
                    ": {\"vcycles\": %d, \"nu_pre\": %d, \"nu_post\": %d, \"mg_precision\": %d, \"mg_tile\": %d, "
                    "\"lanes\": %d, \"ms\": %lf}",
                    &e.vcycles, &e.nu_pre, &e.nu_post, &e.mg_precision, &e.mg_tile, &e.lanes, &e.ms) == 7 ||
        std::sscanf(q1 + 1,
                    ": {\"vcycles\": %d, \"nu_pre\": %d, \"nu_post\": %d, \"mg_precision\": %d, \"mg_tile\": %d, "
                    "\"ms\": %lf}",
                    &e.vcycles, &e.nu_pre, &e.nu_post, &e.mg_precision, &e.mg_tile, &e.ms) == 6)
      m[std::string(q0 + 1, q1)] = e;
  }
  std::fclose(f);
  return m;
}

bool write_cache(const char* path, const std::map<std::string, TuneEntry>& m) {
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return false;
  std::fprintf(f, "{\n");
  size_t k = 0;
  for (const auto& kv : m) {
    const TuneEntry& e = kv.second;
    std::fprintf(f,
                 "  \"%s\": {\"vcycles\": %d, \"nu_pre\": %d, \"nu_post\": %d, \"mg_precision\": %d, \"mg_tile\": %d, "
                 "\"lanes\": %d, \"ms\": %.3f}%s\n",
                 kv.first.c_str(), e.vcycles, e.nu_pre, e.nu_post, e.mg_precision, e.mg_tile, e.lanes, e.ms,
                 ++k < m.size() ? "," : "");
  }
  std::fprintf(f, "}\n");
  const bool ok = std::fclose(f) == 0;
  return ok && std::rename(tmp.c_str(), path) == 0;
}

void apply_entry(const TuneEntry& e, ipmpde_options* o) {
  o->vcycles = e.vcycles;
  o->nu_pre = e.nu_pre;
  o->nu_post = e.nu_post;
  o->mg_precision = e.mg_precision;
  o->mg_tile = e.mg_tile;
  o->lanes = e.lanes;
}

}  // namespace

extern "C" int ipmpde_batch_autotune(ipmpde_batch* B, const ipmpde_options* base, int flags, const char* cache_path,
                                     ipmpde_stream stream, ipmpde_options* best, double* best_ms, int* from_cache) {
  if (!B || !best) return fail(IPMPDE_EINVAL, "NULL argument");
  if (flags & ~IPMPDE_TUNE_PRECISION) return fail(IPMPDE_EINVAL, "unknown autotune flags");
  Group* G = B->G;
  ipmpde_options o;
  TRY(resolve_opts(base, &o));
  if (o.mass_scaling != IPMPDE_MASS_UNIT) return fail(IPMPDE_EINVAL, "the autotuner runs the unit-mass form");
  const std::string key = tune_key(G, o, flags);
  std::map<std::string, TuneEntry> cache;
  if (cache_path) cache = read_cache(cache_path);
  auto hit = cache.find(key);
  if (hit != cache.end()) {
    *best = o;
    apply_entry(hit->second, best);
    TRY(check_options(*best));
    if (best_ms) *best_ms = hit->second.ms;
    if (from_cache) *from_cache = 1;
    return IPMPDE_OK;
  }
  // candidate schedules
  std::vector<TuneEntry> cands;
  const bool p2 = G->dim == 2 && !G->heat &&
                  std::all_of(G->probs.begin(), G->probs.end(), [](const ipmpde_problem* P) {
                    return P->pde == IPMPDE_POISSON || P->pde == IPMPDE_POISSON_Q1;
                  });
  const int precs[2] = {o.mg_precision, o.mg_precision == IPMPDE_FP32 ? IPMPDE_FP64 : IPMPDE_FP32};
  const int nprec = (flags & IPMPDE_TUNE_PRECISION) ? 2 : 1;
  const int sched[5][2] = {{1, 1}, {1, 2}, {1, 3}, {2, 1}, {2, 2}};
  for (int ip = 0; ip < nprec; ++ip)
    for (const auto& vn : sched)
      for (int tile : {IPMPDE_TILE_SMALL, IPMPDE_TILE_LARGE}) {
        if (!p2 && tile == IPMPDE_TILE_LARGE) continue;
        TuneEntry e;
        e.vcycles = vn[0];
        e.nu_pre = e.nu_post = vn[1];
        e.mg_precision = precs[ip];
        e.mg_tile = p2 ? tile : IPMPDE_TILE_AUTO;
        cands.push_back(e);
      }
  const hipStream_t s = S(stream);
  std::vector<ipmpde_options> po(G->count, o);
  int found = 0;
  TuneEntry win;
  // lane counts outermost, so each lane split is built once
  std::vector<TuneEntry> runs;
  for (int L : {1, 2, 4, 8})
    if (L <= G->count)
      for (TuneEntry e : cands) {
        e.lanes = L;
        runs.push_back(e);
      }
  for (TuneEntry& e : runs) {
    for (auto& x : po) apply_entry(e, &x);
    auto solve = [&]() { return e.lanes > 1 ? batch_solve_lanes(B, po, e.lanes, s) : solve_group(G, po, s); };
    // the first solve captures graphs and allocates the precision's levels
    TRY(solve());
    const auto t0 = std::chrono::steady_clock::now();
    TRY(solve());
    e.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    bool ok = true;
    for (const ipmpde_problem* P : G->probs) ok = ok && P->stats.status == IPMPDE_OK;
    if (ok && (!found || e.ms < win.ms)) {
      win = e;
      found = 1;
    }
  }
  if (!found) return fail(IPMPDE_ENOTCONVERGED, "no candidate schedule solved every instance of the batch");
  *best = o;
  apply_entry(win, best);
  if (best_ms) *best_ms = win.ms;
  if (from_cache) *from_cache = 0;
  if (cache_path) {
    cache = read_cache(cache_path);  // keep entries other processes may have added
    cache[key] = win;
    if (!write_cache(cache_path, cache)) return fail(IPMPDE_EINVAL, std::string("cannot write ") + cache_path);
  }
  return IPMPDE_OK;
}
