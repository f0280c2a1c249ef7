// PFTRS without any device allocation (rfp_dpftrs_noalloc): the same kernels
// as rfp_dpftrs (inverses of the factor's 64-row diagonal blocks, then one
// fused substitution per direction), with their scratch in a fixed array of
// the library instead of a handle's workspace.
//
// Scratch layout (one copy per GPU, kept until the process ends):
//   [0, 256)                 control words: [0] epoch of the flags, [1] status
//   [256, 256 + FLAG_BYTES)  ready flags of the fused solves
//   [INV_OFF, SCRATCH_BYTES) inverses of the 64-row diagonal blocks
// Host code never uses the array's name as an address: the device address
// of each GPU's copy is taken once per device with hipGetSymbolAddress and
// kept in a table.
#include <hip/hip_runtime.h>

#include <mutex>

#include "rfp.h"
#include "rfp_common.h"

namespace rfp {

namespace {

constexpr size_t SCRATCH_BYTES = size_t(32) << 20;
constexpr size_t CTL_BYTES = 256;
constexpr size_t FLAG_BYTES = size_t(1) << 20;
constexpr size_t INV_OFF = CTL_BYTES + FLAG_BYTES;
constexpr int64_t MAX_FLAGS = (int64_t)(FLAG_BYTES / sizeof(int));
constexpr int64_t MAX_LEAVES = (int64_t)((SCRATCH_BYTES - INV_OFF) / (sizeof(double) * NB * NB));
constexpr int MAX_DEVICES = 64;

__device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

std::mutex table_mu;
void* table[MAX_DEVICES];  // device address of `scratch` on each device, null until set up

__global__ void clear_ints_kernel(int* p, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0;
}

// Device address of this device's scratch; on the first call on a device
// (with that device current) the address is taken and the control words and
// flags are cleared on `stream`.
hipError_t scratch_of(int dev, hipStream_t stream, unsigned char** out)
{
    std::lock_guard<std::mutex> lock(table_mu);
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    if (!table[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        const int64_t words = (int64_t)((CTL_BYTES + FLAG_BYTES) / sizeof(int));
        hipLaunchKernelGGL(clear_ints_kernel, dim3(256), dim3(256), 0, stream, (int*)p, words);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        table[dev] = p;
    }
    *out = (unsigned char*)table[dev];
    return hipSuccess;
}

}  // namespace

}  // namespace rfp

using namespace rfp;

extern "C" int rfp_dpftrs_noalloc(char transr, char uplo, int64_t n, int64_t nrhs, const double* arf, double* b,
                                  int64_t ldb, hipStream_t stream)
{
    auto upc = [](char c) { return (c >= 'a' && c <= 'z') ? c - 'a' + 'A' : (int)c; };
    if (upc(transr) != 'N' && upc(transr) != 'T') return -1;
    if (upc(uplo) != 'L' && upc(uplo) != 'U') return -2;
    if (n < 0) return -3;
    if (nrhs < 0) return -4;
    if (n > 0 && !arf) return -5;
    if (n > 0 && nrhs > 0 && !b) return -6;
    if (ldb < std::max<int64_t>(1, n)) return -7;
    if (n == 0 || nrhs == 0) return 0;
    RfpBlocks blk;
    rfp_blocks(transr, uplo, n, &blk);
    const int64_t l1 = (blk.m1 + NB - 1) / NB, l2 = (blk.m2 + NB - 1) / NB;
    if (l1 + l2 > MAX_LEAVES || block_solve_flags(blk.m1, blk.m2, nrhs) > MAX_FLAGS) return RFP_ERR_SCRATCH;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return RFP_ERR_RUNTIME;
    unsigned char* base = nullptr;
    if (scratch_of(dev, stream, &base) != hipSuccess) return RFP_ERR_RUNTIME;
    int* ctl = (int*)base;
    int* flags = (int*)(base + CTL_BYTES);
    double* winv = (double*)(base + INV_OFF);
    Exec ex{};
    ex.stream = stream;
    RfpView<const double> v = rfp_view(blk, arf);
    hipError_t e = trtri_leaves<double>(ex, v.t1, blk.m1, winv);
    if (e == hipSuccess) e = trtri_leaves<double>(ex, v.t2, blk.m2, winv + l1 * NB * NB);
    for (int fwd = 1; fwd >= 0 && e == hipSuccess; fwd--) {
        e = epoch_bump(stream, flags, MAX_FLAGS, ctl);
        if (e == hipSuccess)
            e = block_solve<double>(ex, fwd == 1, v.t1, v.s, v.t2, blk.m1, blk.m2, winv, b, ldb, nrhs, flags, ctl,
                                    ctl + 1, DEFAULT_SPIN_LIMIT);
    }
    return e == hipSuccess ? 0 : RFP_ERR_RUNTIME;
}
