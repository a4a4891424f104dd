// The preconditioner apply z = C^{-1} r without a context and without any device
// allocation (aao_apply_Pinv_noalloc in include/aao.h), for callers that cannot
// allocate: code under stream capture, tight serving loops.
//
// Every table and the half spectrum live in one file-scope device array of
// kScratchBytes.  Host code never passes the array's name to a kernel (on the host it
// is only a stand-in): the device address is looked up once per device with
// hipGetSymbolAddress, with that device current, and kept per device.  All calls on
// one device share the array, so calls that overlap in time on one device race.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>

#include "../../include/aao.h"
#include "aao_internal.h"

using namespace aao;

namespace {
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_mu;
unsigned char *g_scratch[kMaxDevices] = {};

size_t up256(size_t b) { return (b + 255) / 256 * 256; }

// device address of `scratch` on the current device `dev` (looked up once)
aao_status scratch_base(int dev, unsigned char **out)
{
    if (dev < 0 || dev >= kMaxDevices) return AAO_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return AAO_ERR_HIP;
        }
        g_scratch[dev] = static_cast<unsigned char *>(p);
    }
    *out = g_scratch[dev];
    return AAO_OK;
}

}  // namespace

extern "C" aao_status aao_apply_Pinv_noalloc(int64_t n, int64_t ell, double tau, double kappa,
                                             int scheme, int prec, const double *r, double *z,
                                             int transpose, void *stream)
{
    if (n < 1 || ell < 2 || !(tau > 0.0) || !std::isfinite(tau) || !(kappa > 0.0) ||
        !std::isfinite(kappa) || !r || !z)
        return AAO_ERR_ARG;
    if (prec != AAO_PREC_FP64 && prec != AAO_PREC_MIXED && prec != AAO_PREC_FP32 &&
        prec != AAO_PREC_MIXED_IN)
        return AAO_ERR_ARG;
    Scheme sc{};
    if (!make_scheme(scheme, tau, &sc)) return AAO_ERR_ARG;
    if (n > 16384 || !fft_supported_fast((int)ell)) return AAO_ERR_UNSUPPORTED;
    const int cfg = solve_default_config((int)n);
    if (cfg < 0) return AAO_ERR_UNSUPPORTED;
    int cw = 0, nt = 0, stg = 0;
    solve_config_shape(cfg, &cw, &nt, &stg);
    const bool sin = prec != AAO_PREC_FP64;
    const bool sout = prec == AAO_PREC_MIXED || prec == AAO_PREC_FP32;
    const bool single_arith = prec == AAO_PREC_FP32;
    const size_t H = (size_t)ell / 2 + 1;
    const int lds = (int)((n + 15) / 16 * 16);
    // layout: twiddles | symbol table | partition tables | half spectrum | the
    // single-precision input spectrum when only the input side is single precision
    const size_t o_tw = 0;
    const size_t o_sym = o_tw + up256(16 * (size_t)ell);
    const size_t o_tab = o_sym + up256(64 * H);
    const size_t o_spec = o_tab + up256(2 * H * (size_t)(3 * cw + 8) * (single_arith ? 8 : 16));
    const size_t o_in = o_spec + up256(H * (size_t)lds * (sout ? 8 : 16));
    const size_t end = o_in + (sin && !sout ? up256(H * (size_t)lds * 8) : 0);
    if (end > kScratchBytes) return AAO_ERR_UNSUPPORTED;
    const size_t N = (size_t)n * (size_t)ell;
    {
        const char *pr = reinterpret_cast<const char *>(r);
        const char *pz = reinterpret_cast<const char *>(z);
        if (pr < pz + 8 * N && pz < pr + 8 * N) return AAO_ERR_ARG;
    }

    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return AAO_ERR_HIP;
    unsigned char *base = nullptr;
    const aao_status s = scratch_base(dev, &base);
    if (s != AAO_OK) return s;
    double *tw = reinterpret_cast<double *>(base + o_tw);
    double *sym = reinterpret_cast<double *>(base + o_sym);
    void *tab = base + o_tab;
    void *spec = base + o_spec;
    void *ispec = sin && !sout ? base + o_in : spec;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int in = (int)n, il = (int)ell;
    // every table is rewritten by this call; the spectrum is fully written by the
    // forward transform before it is read, so nothing has to start at zero
    if (launch_twiddles(tw, il, il, st) != hipSuccess ||
        launch_symbols(sym, in, il, sc, kappa, st) != hipSuccess ||
        launch_solve_tables(sym, in, il, cfg, single_arith, tab, st) != hipSuccess ||
        launch_fft_fwd(r, nullptr, nullptr, nullptr, kappa, in, il, ispec, lds, sin, tw, st, -1,
                       nullptr) != hipSuccess ||
        launch_shifted_solve(ispec, spec, lds, sin, sout, single_arith, in, il, sym, tab,
                             transpose ? 1 : 0, nullptr, st, cfg) != hipSuccess ||
        launch_fft_inv(spec, lds, sout, z, in, il, tw, st, -1, nullptr) != hipSuccess) {
        (void)hipGetLastError();
        return AAO_ERR_HIP;
    }
    return AAO_OK;
}
