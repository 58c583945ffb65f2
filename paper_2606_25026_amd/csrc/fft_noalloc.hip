// Allocation-free 3D transform of a caller's buffer: the transform of the drift
// step (Eq. SPE_solver_KDK (b)) without a plan or workspace, for callers that
// cannot allocate device memory (code under graph capture, serving loops).
//
// Its only device memory beyond the caller's input and output is `scratch`
// below: the descriptor the axis-pass kernels read and the three twiddle
// tables, rewritten by every call.  Each GPU holds its own copy of the array;
// host code reaches it only through the address hipGetSymbolAddress returns
// for the current device (the array's name is a host-side stand-in).
#include <cstring>
#include <mutex>
#include <string>

#include "fft_device.hpp"
#include "wdm.h"
#include "wdm_internal.hpp"

namespace wdm {
void set_last_error(const std::string& msg);
hipError_t launch_scale_complex(hipStream_t s, void* p, int64_t n, double scale, int prec);
}

using namespace wdm;

namespace {

// descriptor (rounded up to 256 bytes) + three tables of at most 512 entries
// of 16 bytes (complex64 hi/lo pairs or complex128 values)
constexpr size_t kDescBytes = (sizeof(MemberDev) + 255) / 256 * 256;
constexpr size_t kTableBytes = 512 * 16;
constexpr size_t kScratchBytes = kDescBytes + 3 * kTableBytes;
static_assert(kScratchBytes <= 32768, "scratch budget");

static __device__ __align__(256) unsigned char scratch[32768];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned char* g_scratch[kMaxDevices] = {};

// Device address of this device's scratch, looked up once per device.
hipError_t scratch_ptr(unsigned char** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch[dev] = static_cast<unsigned char*>(p);
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

// The descriptor arrives as a kernel argument and is stored by one work-group.
__global__ void k_store_desc(MemberDev* __restrict__ dst, MemberDev d) {
    const int words = int(sizeof(MemberDev) / 4);
    const uint32_t* s = reinterpret_cast<const uint32_t*>(&d);
    uint32_t* o = reinterpret_cast<uint32_t*>(dst);
    for (int i = int(threadIdx.x); i < words; i += int(blockDim.x)) o[i] = s[i];
}

// W_n^m = exp(-2 pi i m / n) in FP64; complex64 stores hi = float(w) in
// entries [0, n) and lo = float(w - hi) in [n, 2n), complex128 w itself.
__global__ void k_twiddles(void* __restrict__ dst, int n, int prec) {
    for (int m = int(threadIdx.x); m < n; m += int(blockDim.x)) {
        double s, c;
        sincospi(-2.0 * double(m) / double(n), &s, &c);
        if (prec) {
            static_cast<cplx<double>*>(dst)[m] = cplx<double>{c, s};
        } else {
            cplx<float>* t = static_cast<cplx<float>*>(dst);
            const float hr = float(c), hi = float(s);
            t[m] = cplx<float>{hr, hi};
            t[n + m] = cplx<float>{float(c - double(hr)), float(s - double(hi))};
        }
    }
}

}  // namespace

extern "C" wdm_status wdm_fft3d_noalloc(const void* psi_in, void* psi_out, int32_t nx, int32_t ny,
                                        int32_t nz, int32_t precision, int32_t inverse,
                                        void* hip_stream) {
    auto fail = [](wdm_status st, const std::string& msg) {
        set_last_error(msg);
        return st;
    };
    if (!psi_in || !psi_out) return fail(WDM_EINVAL, "psi_in and psi_out must be non-null");
    if (precision != WDM_C64 && precision != WDM_C128)
        return fail(WDM_EINVAL, "precision must be WDM_C64 or WDM_C128");
    if (!axis_supported(nx) || !axis_supported(ny) || !axis_supported(nz))
        return fail(WDM_EUNSUPPORTED,
                    "axis lengths must be in {16,32,64,96,128,192,256,384,512} (the scratch "
                    "holds twiddle tables of at most 512 entries per axis)");
    const hipStream_t s = static_cast<hipStream_t>(hip_stream);
    unsigned char* base = nullptr;
    hipError_t e = scratch_ptr(&base);
    if (e != hipSuccess)
        return fail(WDM_EDEVICE, std::string("scratch address: ") + hipGetErrorString(e));
    const int prec = precision;
    const int64_t cells = int64_t(nx) * ny * nz;
    MemberDev d;
    std::memset(&d, 0, sizeof(d));
    d.psi = psi_out;
    d.scratch = psi_out;
    d.nx = nx;
    d.ny = ny;
    d.nz = nz;
    unsigned char* tw[3] = {base + kDescBytes, base + kDescBytes + kTableBytes,
                            base + kDescBytes + 2 * kTableBytes};
    d.tw_x = tw[0];
    d.tw_y = tw[1];
    d.tw_z = tw[2];
    MemberDev* desc = reinterpret_cast<MemberDev*>(base);
    const int len[3] = {nx, ny, nz};
    k_store_desc<<<1, 64, 0, s>>>(desc, d);
    for (int a = 0; a < 3; ++a) k_twiddles<<<1, 256, 0, s>>>(tw[a], len[a], prec);
    if ((e = hipGetLastError()) != hipSuccess)
        return fail(WDM_EDEVICE, std::string("set-up launch: ") + hipGetErrorString(e));
    if (psi_in != psi_out &&
        (e = launch_copy_complex(s, psi_out, psi_in, cells, prec, prec)) != hipSuccess)
        return fail(WDM_EDEVICE, std::string("copy: ") + hipGetErrorString(e));
    const Launch L{s, desc, 0, 1};
    const bool inv = inverse != 0;
    // forward: z, y, x; inverse: x, y, z, then the 1/N of the inverse
    for (int k = 0; k < 3; ++k)
        if ((e = launch_axis_fft(L, prec, nx, ny, nz, inv ? k : 2 - k, inv, 0)) != hipSuccess)
            return fail(WDM_EDEVICE, std::string("axis transform: ") + hipGetErrorString(e));
    if (inv && (e = launch_scale_complex(s, psi_out, cells, 1.0 / double(cells), prec)) !=
                   hipSuccess)
        return fail(WDM_EDEVICE, std::string("scale: ") + hipGetErrorString(e));
    return WDM_OK;
}
