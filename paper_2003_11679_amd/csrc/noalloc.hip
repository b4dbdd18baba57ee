// Operator product without device allocation, for callers that cannot
// allocate device memory: code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc.  The stage intermediates of one product
// (grid sources and potentials, FFT pass buffers, per-triangle partials) live
// in a file-scope device array instead of the problem's work buffers.  Each
// device that loads the library holds its own copy of the array until the
// process ends; the host reaches it through the address hipGetSymbolAddress
// returns on that device (the array's name on the host is only a stand-in).
// Every call on one device shares the array: calls that overlap on a device
// race.  Nothing in the product needs the array to start at zero: every
// stage writes all it reads later in the same call.
#include <mutex>

#include "problem.h"
#include "tune.h"

namespace sie {

static __device__ __align__(256) unsigned char scratch[SIE_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static unsigned char *g_scratch[kMaxDevices];
static std::mutex g_scratch_mu;

// Device address of this device's copy of `scratch`, looked up once per
// device with that device current.
void noalloc_init(int device) {
    SIE_CHECK(device >= 0 && device < kMaxDevices, SIE_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch[device]) return;
    int cur = -1;
    SIE_HIP(hipGetDevice(&cur));
    SIE_CHECK(cur == device, SIE_EDEVICE, "scratch lookup needs its device current");
    void *ptr = nullptr;
    SIE_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    SIE_CHECK(ptr != nullptr, SIE_EDEVICE, "no device address for the product scratch");
    g_scratch[device] = static_cast<unsigned char *>(ptr);
}

static int64_t round_up(int64_t b) { return (b + 255) / 256 * 256; }

template <typename T>
static void run(sie_problem *p, Medium &md, sie_op op, const cx<T> *x, cx<T> *y, unsigned char *base,
                hipStream_t st) {
    const ProductSizes n = product_sizes(*md.grid);
    const int64_t es = (int64_t)sizeof(cx<T>);
    const int64_t parts[5] = {n.grid, n.bufA, n.bufB, n.trisrc, n.tripot};
    int64_t need = 0;
    for (int64_t c : parts) need += round_up(c * es);
    SIE_CHECK(need <= (int64_t)SIE_NOALLOC_SCRATCH_BYTES, SIE_EINVAL,
              "medium needs " + std::to_string(need) + " bytes of product scratch, above the " +
                  std::to_string((long long)SIE_NOALLOC_SCRATCH_BYTES) + " the allocation-free product holds");
    cx<T> *ptr[5];
    int64_t off = 0;
    for (int i = 0; i < 5; ++i) {
        ptr[i] = reinterpret_cast<cx<T> *>(base + off);
        off += round_up(parts[i] * es);
    }
    const ProductBufs<T> b{ptr[0], ptr[1], ptr[2], ptr[3], ptr[4]};
    product_one<T>(p, md, op, x, y, b, nullptr, st);
}

void matvec_noalloc(sie_problem *p, Medium &md, sie_op op, sie_precision prec, const void *x, void *y,
                    hipStream_t st) {
    // no launch-shape timing here (it creates events and synchronises):
    // shapes already tuned are used, else the built-in ones
    TuneSuspend no_tuning;
    int cur = -1;
    SIE_HIP(hipGetDevice(&cur));
    SIE_CHECK(cur == p->ctx->device, SIE_EDEVICE, "the problem's device must be current");
    unsigned char *base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        base = g_scratch[cur];
    }
    SIE_CHECK(base != nullptr, SIE_ESTATE, "product scratch not looked up on this device");
    if (op == SIE_OP_X) {
        // the X product has no intermediates
        if (prec == SIE_FP64)
            launch_x_apply<double>(p->mesh.nrwg, p->d_xptr.p, p->d_xcol.p, p->d_xval64.p, (const c128 *)x, (c128 *)y,
                                   st);
        else
            launch_x_apply<float>(p->mesh.nrwg, p->d_xptr.p, p->d_xcol.p, p->d_xval32.p, (const c64 *)x, (c64 *)y,
                                  st);
        return;
    }
    if (prec == SIE_FP64) run<double>(p, md, op, (const c128 *)x, (c128 *)y, base, st);
    else run<float>(p, md, op, (const c64 *)x, (c64 *)y, base, st);
}

}  // namespace sie
