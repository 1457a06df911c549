// Allocation-free variant of the library's GEMM entry point.
//
// gpqmc_debug_gemm builds the GEMM descriptor (one GemmEntry and the output
// tile list) in device memory it allocates per call.  gpqmc_gemm_noalloc keeps
// them in the file-scope array `scratch` instead, a fixed block of device
// memory that every GPU the library runs on holds until the process ends, and
// has a one-workgroup kernel write them from its arguments, so the call makes
// no allocation and no host-to-device copy and can be captured in a HIP graph.
// Host code reaches the array only through the address hipGetSymbolAddress
// returns for the current device (kept per device); the name itself is a
// host-side stand-in, not a device address.
#include <hip/hip_runtime.h>

#include <cstring>

#include "../../include/gpqmc.h"
#include "gpqmc_internal.h"

namespace gpqmc {
hipError_t launch_gemm_l(int mode, const GemmEntry* e, const TileRef* t, int n, GemmArgs a,
                         hipStream_t s);
hipError_t launch_gemm_l64(int mode, const GemmEntry* e, const TileRef* t, int n, GemmArgs a,
                           hipStream_t s);
hipError_t launch_gemm_plain(int fp32, int transA, const GemmEntry* e, const TileRef* t, int n,
                             GemmArgs a, hipStream_t s);
}  // namespace gpqmc

using namespace gpqmc;

namespace {

constexpr size_t kScratchBytes = 256 * 1024;   // GemmEntry + up to 16352 output tiles
constexpr size_t kTileOffset = 512;            // TileRef list after the entry (512-byte slot)
constexpr int kMaxTiles = (int)((kScratchBytes - kTileOffset) / sizeof(TileRef));
constexpr int kMaxDevices = 64;
static_assert(sizeof(GemmEntry) <= kTileOffset, "the entry fits before the tile list");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

void* g_scratch_ptr[kMaxDevices] = {nullptr};   // per device, from hipGetSymbolAddress

// Writes the GEMM descriptor into the scratch block: the entry (every field,
// so nothing of an earlier call survives) and the row-major list of output
// tiles of a tm x tn grid.
__global__ void k_fill_gemm_desc(unsigned char* scr, const void* A, const void* B, void* C, int M,
                                 int N, int K, int lda, int ldb, int ldc, int tm, int tn) {
  GemmEntry* e = reinterpret_cast<GemmEntry*>(scr);
  TileRef* t = reinterpret_cast<TileRef*>(scr + kTileOffset);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    GemmEntry v;
    unsigned char* raw = reinterpret_cast<unsigned char*>(&v);
    for (size_t i = 0; i < sizeof v; ++i) raw[i] = 0;
    v.A[0] = v.A[1] = A;
    v.B[0] = v.B[1] = B;
    v.C[0] = v.C[1] = C;
    v.M = M;
    v.N = N;
    v.K = K;
    v.lda = lda;
    v.ldb = ldb;
    v.ldc = ldc;
    *e = v;
  }
  const int n = tm * tn;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    t[i] = TileRef{0, i / tn, i % tn, 0};
}

}  // namespace

extern "C" gpqmc_status gpqmc_gemm_noalloc(int32_t precision, int32_t M, int32_t N, int32_t K,
                                           int32_t flags, const void* A, int32_t lda, const void* B,
                                           int32_t ldb, void* C, int32_t ldc, void* hip_stream) {
  if (M <= 0 || N <= 0 || K < 0 || !A || !B || !C) return GPQMC_EINVAL;
  const int trans_a = flags & 1, large = (flags >> 1) & 1;
  if ((flags & ~3) || (precision != GPQMC_MIXED && precision != GPQMC_FP64) || (large && trans_a))
    return GPQMC_EINVAL;
  const int tile = large ? 128 : kTile;
  const long long tm = (M + tile - 1) / tile, tn = (N + tile - 1) / tile;
  if (tm * tn > kMaxTiles) return GPQMC_EINVAL;   // beyond the scratch block's tile list
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return GPQMC_EHIP;
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return GPQMC_EHIP;
    g_scratch_ptr[dev] = p;
  }
  unsigned char* scr = static_cast<unsigned char*>(g_scratch_ptr[dev]);
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const int nt = (int)(tm * tn);
  hipLaunchKernelGGL(k_fill_gemm_desc, dim3((nt + 255) / 256), dim3(256), 0, s, scr, A, B, C, M, N,
                     K, lda, ldb, ldc, (int)tm, (int)tn);
  if (hipGetLastError() != hipSuccess) return GPQMC_EHIP;
  const GemmEntry* e = reinterpret_cast<const GemmEntry*>(scr);
  const TileRef* t = reinterpret_cast<const TileRef*>(scr + kTileOffset);
  GemmArgs a;
  memset(&a, 0, sizeof a);
  a.scale_slice = -1;
  a.bscale_slice = -1;
  hipError_t err;
  if (large && precision == GPQMC_MIXED)
    err = launch_gemm_l(GM_STORE, e, t, nt, a, s);
  else if (large)
    err = launch_gemm_l64(GM_STORE, e, t, nt, a, s);
  else
    err = launch_gemm_plain(precision == GPQMC_MIXED, trans_a, e, t, nt, a, s);
  return err == hipSuccess ? GPQMC_OK : GPQMC_EHIP;
}
