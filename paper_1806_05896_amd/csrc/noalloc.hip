// Entry points that allocate nothing, for callers that cannot call the
// device allocator (code under stream capture, tight serving loops,
// harnesses that forbid allocation).  Their scratch memory is one
// file-scope device array per GPU; its device address is looked up once per
// device with hipGetSymbolAddress and only that address is handed to
// kernels and copies (the array's name is a host-side stand-in in host
// code).  Every call on a GPU shares that GPU's array, so calls that overlap
// on one GPU race; each call sets up what it needs (the ticket counters are
// cleared by a fill kernel, the descriptor copied in) before its kernels run.

namespace {

constexpr size_t kScratchBytes = size_t(4) << 20;      // 4 MiB per GPU
constexpr size_t kScrDesc = 0;                         // launch descriptor (Inst)
constexpr size_t kScrCounter = 4096;                   // reduction ticket counters
constexpr size_t kScrStat = kScrCounter + 4096;        // results (16 doubles)
constexpr size_t kScrPartials = kScrStat + 256;        // per-block partials of the reduction
constexpr int kScratchDevices = 64;
static_assert(sizeof(ipm::Inst) <= kScrCounter - kScrDesc, "descriptor area too small");
static_assert(sizeof(unsigned) * ipm::kTicketStride * (ipm::kTicketGroups + 1) <= kScrStat - kScrCounter,
              "ticket area too small");

std::mutex g_scratch_mu;
void* g_scratch_dev[kScratchDevices];  // device address of `scratch` on each GPU (null: not looked up)

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace ipm {
__global__ void __launch_bounds__(256) k_zero_words(unsigned* __restrict__ p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0u;
}
}  // namespace ipm

// Device address of this GPU's scratch array (the current device's).
static int scratch_base(char** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kScratchDevices) return fail(IPMPDE_EDEVICE, "device index out of range for the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(IPMPDE_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_dev[dev] = p;
  }
  *out = (char*)g_scratch_dev[dev];
  return IPMPDE_OK;
}

// Largest n whose reduction partials fit: whole groups of 8 blocks of kBS
// nodes, three partials each (44,648,448 nodes with 4 MiB).
static size_t noalloc_max_nodes() {
  return (((kScratchBytes - kScrPartials) / (3 * sizeof(double))) & ~size_t(7)) * kBS;
}

extern "C" int ipmpde_measures_noalloc(ipmpde_problem* P, ipmpde_stream stream, double* xp, double* xd, double* xc) {
  if (!P || !xp || !xd || !xc) return fail(IPMPDE_EINVAL, "NULL argument");
  if (P->in_engine) return fail(IPMPDE_EINVAL, "problem is queued or running in an engine");
  if (P->need_init)
    return fail(IPMPDE_EINVAL, "iterates not set: call ipmpde_reset or ipmpde_solve first (they allocate)");
  const int nb = nblk((long)P->n);
  const size_t need = kScrPartials + 3 * (size_t)nb * sizeof(double);
  if (need > kScratchBytes)
    return fail(IPMPDE_EINVAL, "problem too large for ipmpde_measures_noalloc: " + std::to_string(P->n) +
                                   " nodes, at most " + std::to_string(noalloc_max_nodes()));
  char* base = nullptr;
  TRY(scratch_base(&base));
  Inst d = P->I;
  d.active = 1;
  d.counter = (unsigned*)(base + kScrCounter);
  d.stat = (double*)(base + kScrStat);
  d.partials = (double*)(base + kScrPartials);
  d.nparts = 3 * nb;
  const hipStream_t s = S(stream);
  HIP_TRY(hipMemcpyAsync(base + kScrDesc, &d, sizeof(Inst), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(256), 0, s, d.counter, kTicketStride * (kTicketGroups + 1));
  hipLaunchKernelGGL(k_measures, dim3(nb, 1, 1), dim3(kBS), 0, s, (const Inst*)(base + kScrDesc));
  HIP_TRY(hipGetLastError());
  double r[3];
  HIP_TRY(hipMemcpyAsync(r, d.stat, sizeof(r), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));  // also keeps d alive until its copy has been consumed
  *xp = P->rep * r[0];
  *xd = P->rep * r[1];
  *xc = P->rep * r[2];
  return IPMPDE_OK;
}
