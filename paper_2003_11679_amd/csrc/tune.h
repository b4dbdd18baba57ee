// Launch-shape tuner for the grid stages: the FFT passes' tile shapes
// (threads and values per thread of a block, which set the lines per LDS
// tile) and the block sizes of projection and interpolation.  Every
// candidate of a family computes the same values with the same arithmetic
// (only the mapping of work onto threads differs), so a choice never
// changes a result, only the time.
//
// On the first launch of a family for a given problem shape, the candidates
// are timed on the caller's stream (HIP events, one warm-up and three timed
// launches each) and the fastest is kept for the rest of the process (per
// device).  Tuning is skipped, and the first candidate (the built-in shape)
// used, when it is switched off, while the stream is being captured into a
// graph, under TuneSuspend, or while another thread is tuning.
#pragma once

#include <functional>
#include <string>

#include "common.h"

namespace sie {

enum TuneFamily {
    TUNE_FFT_YFWD = 0,   // forward pass along y (strided lines)
    TUNE_FFT_YINV = 1,   // inverse pass along y
    TUNE_FFT_Z = 2,      // fused z pass with the G spectrum
    TUNE_PROJECT = 3,    // projection (threads per block)
    TUNE_INTERP = 4,     // interpolation (threads per block)
    TUNE_NFAMILY = 5
};

struct TuneKey {
    int device = 0;
    int family = 0;
    int prec = 0;        // bytes per real
    int64_t d[5] = {0, 0, 0, 0, 0};
    bool operator<(const TuneKey &o) const;
};

// 0: built-in shapes only; 1: tune on first use (default).
void tune_set_mode(int mode);
int tune_get_mode();
// Testing: always use candidate `c` of `family` (-1: back to tuning).
void tune_force(int family, int c);

// Candidate to use for key k among ncand: run(c) launches candidate c on
// st, or returns false without launching when c does not apply to this
// shape (candidate 0 always applies).  Times the candidates on the first
// call for k (see above).
int tune_pick(const TuneKey &k, int ncand, const std::function<bool(int)> &run, hipStream_t st);
// Cached choice for k without tuning (the forced one, else 0 when none).
int tune_cached(const TuneKey &k);

// While one is alive on a host thread, that thread never tunes.
struct TuneSuspend {
    TuneSuspend();
    ~TuneSuspend();
    TuneSuspend(const TuneSuspend &) = delete;
    TuneSuspend &operator=(const TuneSuspend &) = delete;
};

// One line per tuned key: family, precision, shape, candidate times (us) and
// the choice.
std::string tune_report();
void tune_clear();

}  // namespace sie
