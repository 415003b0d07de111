// Allocation-free form of the whole hot path (sfft_run_noalloc).
//
// Every device buffer the path needs beyond the caller's inputs and outputs
// -- the workspace of one geometry (row / column spectra, lag rows, lag
// tables, normal matrix, factor, solve flags) and the twiddle tables of both
// line lengths -- is carved from one file-scope device array, `scratch`, of
// kScratchBytes. Host code never passes the array's name to a kernel (on the
// host it is only a stand-in symbol): its device address is taken once per
// device with hipGetSymbolAddress and kept in scratch_ptr[device].
#include <hip/hip_runtime.h>

#include <mutex>

#include "runtime.hpp"

namespace sfft {

constexpr size_t kScratchBytes = size_t(128) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kScratchBytes];

static std::mutex scratch_mu;
static char* scratch_ptr[kMaxDevices];

// Device address of `scratch` on `device` (taken once, with that device
// current). Returns SFFT_OK or SFFT_E_HIP.
int noalloc_init(int device) {
    if (device < 0 || device >= kMaxDevices) return SFFT_E_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (scratch_ptr[device]) return SFFT_OK;
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return SFFT_E_HIP;
    if (cur != device && hipSetDevice(device) != hipSuccess) return SFFT_E_HIP;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess || !ptr) return SFFT_E_HIP;
    scratch_ptr[device] = static_cast<char*>(ptr);
    return SFFT_OK;
}

static char* noalloc_ptr(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(scratch_mu);
    return scratch_ptr[device];
}

// Twiddle tables of one line plan, formed on the device (the same entries
// make_twiddles forms on the host): tw[t] = e^(-2 pi i t / n), the pass
// tables (pass p >= 1 of radix R after ns = product of the earlier radices:
// row k holds W_(ns R)^(r k) for r < R, 16 entries per row, zero elsewhere),
// and twp = cos, sin of +2 pi t / n in FP64.
template <typename T>
__global__ void twiddle_kernel(LinePlan lp, int tlen, cx<T>* __restrict__ tw,
                               cx<T>* __restrict__ twt, double* __restrict__ twp) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = lp.n;
    if (i < n) {
        double sn, cs;
        sincospi(2.0 * (double)i / (double)n, &sn, &cs);
        tw[i] = mk(T(cs), T(-sn));
        twp[2 * i] = cs;
        twp[2 * i + 1] = sn;
    }
    if (i < tlen) {
        cx<T> v = mk(T(0), T(0));
        int ns = lp.radix[0];
        for (int p = 1; p < lp.npass; ++p) {
            const int R = lp.radix[p], off = lp.twoff[p];
            if (i >= off && i < off + ns * 16) {
                const int k = (i - off) >> 4, r = (i - off) & 15;
                if (r < R) {
                    const long long den = (long long)ns * R;
                    const long long num = ((long long)r * k) % den;
                    double sn, cs;
                    sincospi(2.0 * (double)num / (double)den, &sn, &cs);
                    v = mk(T(cs), T(-sn));
                }
            }
            ns *= R;
        }
        twt[i] = v;
    }
}

template <typename T>
static hipError_t fill_twiddles(const LinePlan& lp, const Twiddles& t, hipStream_t st) {
    const int tlen = pass_table_len(lp.n) + 16;
    const int cnt = lp.n > tlen ? lp.n : tlen;
    hipLaunchKernelGGL(twiddle_kernel<T>, dim3((cnt + 255) / 256), dim3(256), 0, st, lp, tlen,
                       static_cast<cx<T>*>(t.tw), static_cast<cx<T>*>(t.twt), t.twp);
    return hipGetLastError();
}

// Twiddle tables of length n carved after the workspace (nullptr base:
// sizes only).
static void carve_twiddles(Carver& c, char* base, int n, size_t cxb, Twiddles& t) {
    t.tw = c.take<char>(base, cxb * (size_t)n);
    t.twt = c.take<char>(base, cxb * (size_t)(pass_table_len(n) + 16));
    t.twp = c.take<double>(base, 2 * (size_t)n);
}

// Workspace plus twiddles of `p` carved from `base` (nullptr: sizes only);
// returns the bytes used.
static size_t carve_all(Plan& pl, char* base) {
    const bool mixed = pl.p.precision == SFFT_MIXED;
    const size_t cxb = mixed ? 8 : 16;
    Carver c;
    c.off = carve(pl.ws, pl.g, cxb, mixed ? 4 : 8, base);
    carve_twiddles(c, base, pl.p.n0, cxb, pl.t0);
    if (pl.p.n1 == pl.p.n0)
        pl.t1 = pl.t0;
    else
        carve_twiddles(c, base, pl.p.n1, cxb, pl.t1);
    return c.off + 256;
}

int run_noalloc(int device, const sfft_params* p, const void* rf, const void* sf, const void* r,
                const void* s, double* coef, void* d, hipStream_t st) {
    int rc = check_params(p);
    if (rc) return rc;
    char* base = noalloc_ptr(device);
    if (!base) return SFFT_E_HIP;
    Plan pl;
    pl.p = *p;
    pl.g = make_geom(p);
    pl.lp0 = make_line_plan(p->n0);
    pl.lp1 = make_line_plan(p->n1);
    // lengths that need Bluestein tables (formed on the host) are not served here
    if (pl.lp0.nl != pl.lp0.n || pl.lp1.nl != pl.lp1.n) return SFFT_E_UNSUPPORTED;
    pl.device = device;
    if (carve_all(pl, nullptr) > kScratchBytes) return SFFT_E_NOMEM;
    carve_all(pl, base);
    pl.ws.base = base;
    pl.ws.bytes = kScratchBytes;
    const bool mixed = p->precision == SFFT_MIXED;
    hipError_t e = mixed ? fill_twiddles<float>(pl.lp0, pl.t0, st) : fill_twiddles<double>(pl.lp0, pl.t0, st);
    if (!e && p->n1 != p->n0)
        e = mixed ? fill_twiddles<float>(pl.lp1, pl.t1, st) : fill_twiddles<double>(pl.lp1, pl.t1, st);
    if (!e) e = launch_polysum(pl.g, poly_degree(pl.g), pl.ws.sig0, pl.ws.sig1, pl.ws.pw, st);
    if (e) return SFFT_E_HIP;
    rc = plan_run(pl, rf, sf, r, s, coef, d, st);
    if (rc || st) return rc;
    // synchronous mode: the device status of this call
    int f = 0;
    if (hipStreamSynchronize(nullptr) != hipSuccess ||
        hipMemcpy(&f, pl.ws.flag, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
        return SFFT_E_HIP;
    return flag_status(f);
}

}  // namespace sfft
