// Launch-shape tuner (tune.h).
#include "tune.h"

#include <atomic>
#include <map>
#include <mutex>
#include <sstream>
#include <tuple>
#include <vector>

namespace sie {

bool TuneKey::operator<(const TuneKey &o) const {
    return std::tie(device, family, prec, d[0], d[1], d[2], d[3], d[4]) <
           std::tie(o.device, o.family, o.prec, o.d[0], o.d[1], o.d[2], o.d[3], o.d[4]);
}

namespace {

struct Entry {
    int choice = 0;
    std::vector<float> us;   // per candidate
};

struct Tuner {
    std::mutex mu;                     // guards the table
    std::mutex busy;                   // held while a thread times candidates
    std::map<TuneKey, Entry> table;
    std::atomic<int> mode{1};
    std::atomic<int> forced[TUNE_NFAMILY];
    Tuner() {
        for (auto &f : forced) f.store(-1);
    }
};

Tuner &tuner() {
    static Tuner *t = new Tuner;
    return *t;
}

thread_local int t_suspended = 0;

const char *family_name(int f) {
    switch (f) {
        case TUNE_FFT_YFWD: return "fft_y_fwd";
        case TUNE_FFT_YINV: return "fft_y_inv";
        case TUNE_FFT_Z: return "fft_z";
        case TUNE_PROJECT: return "project";
        case TUNE_INTERP: return "interp";
        default: return "?";
    }
}

}  // namespace

TuneSuspend::TuneSuspend() { ++t_suspended; }
TuneSuspend::~TuneSuspend() { --t_suspended; }

void tune_set_mode(int mode) {
    SIE_CHECK(mode == 0 || mode == 1, SIE_EINVAL, "tuning mode must be 0 or 1");
    tuner().mode.store(mode);
}
int tune_get_mode() { return tuner().mode.load(); }

void tune_force(int family, int c) {
    SIE_CHECK(family >= 0 && family < TUNE_NFAMILY, SIE_EINVAL, "unknown tuning family");
    SIE_CHECK(c >= -1, SIE_EINVAL, "candidate index below -1");
    tuner().forced[family].store(c);
}

int tune_cached(const TuneKey &k) {
    Tuner &T = tuner();
    const int f = T.forced[k.family].load();
    if (f >= 0) return f;
    std::lock_guard<std::mutex> lk(T.mu);
    auto it = T.table.find(k);
    return it == T.table.end() ? 0 : it->second.choice;
}

int tune_pick(const TuneKey &k, int ncand, const std::function<bool(int)> &run, hipStream_t st) {
    Tuner &T = tuner();
    const int f = T.forced[k.family].load();
    if (f >= 0) {
        SIE_CHECK(f < ncand, SIE_EINVAL, std::string("forced candidate out of range for ") + family_name(k.family));
        return f;
    }
    {
        std::lock_guard<std::mutex> lk(T.mu);
        auto it = T.table.find(k);
        if (it != T.table.end()) return it->second.choice;
    }
    if (ncand <= 1 || T.mode.load() == 0 || t_suspended) return 0;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    SIE_HIP(hipStreamIsCapturing(st, &cap));
    if (cap != hipStreamCaptureStatusNone) return 0;
    std::unique_lock<std::mutex> busy(T.busy, std::try_to_lock);
    if (!busy.owns_lock()) return 0;
    Entry e;
    e.us.assign(ncand, 0.0f);
    hipEvent_t a = nullptr, b = nullptr;
    SIE_HIP(hipEventCreate(&a));
    try {
        SIE_HIP(hipEventCreate(&b));
        constexpr int kReps = 3;
        for (int c = 0; c < ncand; ++c) {
            if (!run(c)) {   // warm-up (code load, caches); or not applicable
                e.us[c] = -1.0f;
                continue;
            }
            SIE_HIP(hipEventRecord(a, st));
            for (int r = 0; r < kReps; ++r) run(c);
            SIE_HIP(hipEventRecord(b, st));
            SIE_HIP(hipEventSynchronize(b));
            float ms = 0.0f;
            SIE_HIP(hipEventElapsedTime(&ms, a, b));
            e.us[c] = 1000.0f * ms / kReps;
            if (e.us[c] < e.us[e.choice]) e.choice = c;
        }
    } catch (...) {
        (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
        throw;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    std::lock_guard<std::mutex> lk(T.mu);
    T.table[k] = e;
    return e.choice;
}

std::string tune_report() {
    Tuner &T = tuner();
    std::lock_guard<std::mutex> lk(T.mu);
    std::ostringstream os;
    for (const auto &kv : T.table) {
        const TuneKey &k = kv.first;
        os << family_name(k.family) << " dev=" << k.device << " fp" << 8 * k.prec << " shape=";
        for (int i = 0; i < 5; ++i) os << (i ? "x" : "") << k.d[i];
        os << " us=";
        for (size_t c = 0; c < kv.second.us.size(); ++c) os << (c ? "," : "") << kv.second.us[c];
        os << " choice=" << kv.second.choice << "\n";
    }
    return os.str();
}

void tune_clear() {
    Tuner &T = tuner();
    std::lock_guard<std::mutex> lk(T.mu);
    T.table.clear();
}

}  // namespace sie
