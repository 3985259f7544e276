// Extraction that allocates nothing: the variant of tc_extract for callers
// that cannot allocate device memory (code under stream capture, tight
// serving loops, harnesses that forbid it).  Its launch descriptor, step
// state, indenter poses, tile lists and partial sums live in one file-scope
// device array of fixed size instead of the context's step scratch, plan and
// state pool; the kernels are the ones tc_extract launches.
#include <mutex>

#include "runtime.h"

namespace tc {
namespace {

constexpr size_t NOALLOC_BYTES = size_t(4) << 20;   // TC_NOALLOC_SCRATCH_BYTES
constexpr int MAX_DEVICES = 64;
static_assert(NOALLOC_BYTES == TC_NOALLOC_SCRATCH_BYTES, "header and library agree on the size");

// One copy per device.  Host code never passes this name to a kernel or a
// copy: it takes the device address from hipGetSymbolAddress below.
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

std::mutex g_mu;
void* g_ptr[MAX_DEVICES] = {};

size_t up256(size_t b) { return (b + 255) & ~size_t(255); }
int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// Tile list {pad 0, tile i} for i < n.
__global__ void k_noalloc_tiles(Tile* t, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) t[i] = Tile{0, i};
}

}  // namespace

// Device address of this device's scratch array, looked up once per device
// with that device current (context creation).
tc_status noalloc_init(int device) {
  if (device < 0 || device >= MAX_DEVICES) return set_error(TC_E_INVALID_ARG, "device ordinal beyond 63");
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[device]) return TC_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(no-alloc scratch)");
  if (!p) return set_error(TC_E_HIP, "no-alloc scratch has no device address");
  g_ptr[device] = p;
  return TC_OK;
}

}  // namespace tc

using namespace tc;

tc_status tc_extract_noalloc(tc_pad* pad, int32_t n_ind, const tc_indenter* ind, double* reaction) {
  if (!pad) return set_error(TC_E_INVALID_ARG, "pad is null");
  tc_context* ctx = pad->ctx;
  std::string err;
  tc_status s = validate_indenters(n_ind, ind, err);
  if (s) return set_error(s, err);
  if ((s = check_meshes(ctx, n_ind, ind))) return s;
  if (pad->busy.load()) return set_error(TC_E_BUSY, "pad has a request in flight on a server");
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  TC_HIP(hipSetDevice(ctx->device));
  char* base;
  {
    std::lock_guard<std::mutex> g(g_mu);
    base = ctx->device < MAX_DEVICES ? static_cast<char*>(g_ptr[ctx->device]) : nullptr;
  }
  if (!base) return set_error(TC_E_HIP, "no-alloc scratch not initialised on this device");
  // layout: descriptor, state, poses, tiles (tet, surface, contact vertex),
  // contact and traction partial sums
  const int n_tt = cdiv(pad->T, ctx->el_block);
  const int n_st = cdiv(pad->S, ctx->cg_block);
  const int n_ct = pad->C > 0 ? cdiv(pad->C, ctx->cg_block) : 0;
  size_t off = 0;
  auto take = [&](size_t b) { const size_t o = off; off += up256(b); return o; };
  const size_t o_desc = take(sizeof(EnvDesc));
  const size_t o_state = take(sizeof(EnvState));
  const size_t o_pose = take(sizeof(EnvPose));
  const size_t o_tiles = take(sizeof(Tile) * ((size_t)n_tt + n_st + n_ct));
  const size_t o_c3 = take(24 * (size_t)std::max(n_ct, 1));
  const size_t o_s3 = take(24 * (size_t)std::max(n_st, 1));
  if (off > NOALLOC_BYTES)
    return set_error(TC_E_INVALID_ARG, "pad needs " + std::to_string(off) + " bytes of no-alloc scratch, more than " +
                                           std::to_string(NOALLOC_BYTES));
  EnvDesc E = pad->desc;
  E.n_tt = n_tt;
  E.n_st = n_st;
  E.n_ct = n_ct;
  E.part_c3 = reinterpret_cast<double*>(base + o_c3);
  E.part_s3 = reinterpret_cast<double*>(base + o_s3);
  E.st = reinterpret_cast<EnvState*>(base + o_state);
  E.pose = reinterpret_cast<const EnvPose*>(base + o_pose);
  EnvState S;
  EnvPose Q;
  init_state(S, Q, 1, n_ind, ind, pad);
  if (Q.pairs)
    return set_error(TC_E_INVALID_ARG,
                     "vertex-face / edge-edge pairs (mesh_contact 2 with a mesh indenter) need the pad's step "
                     "scratch: use tc_extract");
  hipStream_t st = ctx->stream;
  TC_HIP(hipMemcpyAsync(base + o_desc, &E, sizeof E, hipMemcpyHostToDevice, st));
  TC_HIP(hipMemcpyAsync(base + o_state, &S, sizeof S, hipMemcpyHostToDevice, st));
  TC_HIP(hipMemcpyAsync(base + o_pose, &Q, sizeof Q, hipMemcpyHostToDevice, st));
  Tile* tiles = reinterpret_cast<Tile*>(base + o_tiles);
  Tile* t_tet = tiles;
  Tile* t_surf = tiles + n_tt;
  Tile* t_cand = tiles + n_tt + n_st;
  const int counts[3] = {n_tt, n_st, n_ct};
  Tile* lists[3] = {t_tet, t_surf, t_cand};
  for (int c = 0; c < 3; ++c)
    if (counts[c] > 0) hipLaunchKernelGGL(k_noalloc_tiles, dim3(cdiv(counts[c], 256)), dim3(256), 0, st, lists[c], counts[c]);
  const EnvDesc* d_desc = reinterpret_cast<const EnvDesc*>(base + o_desc);
  auto go = [&](KernelId k, const Tile* t, int nt, int block) {
    LaunchArgs a;
    a.envs = d_desc;
    a.n_env = 1;
    a.stream = st;
    a.tiles = t;
    a.ntiles = nt;
    a.block = block;
    return launch_kernel(k, pad->fp64, a);
  };
  (void)go(KernelId::sigma, t_tet, n_tt, ctx->el_block);
  (void)go(KernelId::traction, t_surf, n_st, ctx->cg_block);
  (void)go(KernelId::contact, t_cand, n_ct, ctx->cg_block);
  (void)go(KernelId::env_extract, nullptr, 0, 256);
  TC_HIP(hipGetLastError());
  TC_HIP(hipMemcpyAsync(&S, base + o_state, sizeof S, hipMemcpyDeviceToHost, st));
  TC_HIP(hipStreamSynchronize(st));
  if (S.status != TC_OK) return set_error(S.status, "extraction failed");
  if (reaction)
    for (int c = 0; c < 3; ++c) reaction[c] = S.reaction[c];
  return TC_OK;
}
