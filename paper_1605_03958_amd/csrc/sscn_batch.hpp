// sscn_batch.hpp -- device-resident instance table and work list of the
// batched persistent SSCN step (sscn_batch.hip, sscn_batch_api.cpp).
//
// Every step is one launch of k_batch_step.  Its blocks take work items in
// ticket order from a list built on the host in dependency order: all x-line
// tiles of all instances, then y, then z, then the observation tiles, then
// one finalisation item per instance.  An item waits (bounded spin) until
// its instance's previous pass has completed all its tiles; every item waits
// only for items with smaller tickets, which running blocks already hold, so
// the waits always end.  The last block to leave resets the counters, so the
// next launch (or graph replay) starts clean.  Tile shapes depend only on an
// instance's own shape and every reduction has fixed slots and a fixed
// order: an instance's results do not depend on what else is in the batch.
//
// A 1D instance whose line fits one block is a solo instance: one item runs
// its whole step (line solve, observation sums, finalisation) inside one
// block, with block barriers in place of the counters, and repeats steps
// while other items of the launch are still unclaimed (at least
// BCtl::solo_min and at most BATCH_SOLO_MAX steps per launch).  While every
// instance of the batch is solo, a launch is k_batch_solo instead: one block
// per instance, BATCH_SOLO_ONLY steps with the line held in registers.  In a
// mixed batch on a stream, one launch of the same kernel per sscn_batch_step
// call runs the solo instances on a second stream beside that call's
// persistent launches (which leave them out of their work list, and whose
// grid leaves their CUs free), stepping until the last of those launches has
// finished (the persistent kernel counts its launches in reg_epoch), and at
// least once.  The
// line solve, the observation sums and the finalisation are the same
// arithmetic either way, so only the number of steps a launch advances an
// instance varies.
#pragma once

#include <stdint.h>

#include "sscn_dev.hpp"
#include "sscn_launch.hpp"

namespace sscn {

enum { BP_X = 0, BP_Y = 1, BP_Z = 2, BP_OBS = 3, BP_FIN = 4, BP_NPASS = 5, BP_SOLO = 5 };
enum { BS_EMPTY = 0, BS_RUNNING = 1, BS_CONVERGED = 2, BS_DONE = 3, BS_NONFINITE = 4, BS_STALLED = 5 };

constexpr int BATCH_BLOCK = 1024;     // threads per block of the persistent kernel
constexpr int BATCH_LDS = 64 * 1024;  // dynamic LDS bytes of every persistent block
constexpr int BATCH_OBS_PTS = 16384;  // grid points per observation tile, at least
constexpr int BATCH_NOBS = 10;        // FP64 sums per observation tile
constexpr int BATCH_SOLO_MAX = 256;   // steps of a solo instance per launch, at most
constexpr int BATCH_SOLO_ONLY = 64;   // ... and at least, once only solo instances run
constexpr int BATCH_SOLO_HEAD = 1024; // table head entries (i < i_conv) of a register-resident solo line, at most

// Geometry of one axis of one instance (see sscn_lines.hpp for ROW / COL).
struct BAxis {
    int32_t kind;      // K_ROW (x) or K_COL (y, z)
    int32_t C;         // points per thread
    int32_t wpl;       // ROW: waves per line
    int32_t lpi;       // ROW: lines per item (16 / wpl)
    int32_t W, L;      // COL: waves and lanes per line of one sub-tile
    int32_t tpi;       // COL: sub-tiles per item (16 / W)
    int32_t rep;       // line groups (ROW) or sub-tile sets (COL) per item
    int32_t ntiles;    // items of this pass
    int64_t nlines;
    int64_t stride;
    int64_t s1, s2;
    int32_t m1;
    double sig_re, sig_im;
    LineTab lt;        // table in the instance workspace
};

// Static description of an admitted instance (host-written at admission).
struct BInst {
    void *psi;
    int32_t elem;          // 1 float (imaginary time), 3 complex<float> (real time)
    int32_t dim;
    int64_t npts;
    PointParams pp;
    BAxis ax[3];
    double *norm_part;     // one FP64 per tile of the last sweep
    double *obs_part;      // BATCH_NOBS FP64 per observation tile
    int32_t obs_tiles;
    int64_t obs_pts;       // grid points per observation tile
    int32_t observe_every;
    double mu_tol;         // > 0: stop at |mu - mu_prev| < mu_tol between observations
    int64_t max_steps;
    double dvol;
    int32_t imag;
    int32_t last_pass;     // BP_X + dim - 1
    int32_t dep[BP_NPASS]; // pass an item of this pass waits for (-1: none)
    int32_t need[BP_NPASS];// tiles of that pass
    int32_t solo;          // whole step in one item (1D, one line, one observation tile)
};

// Dynamic per-instance state (device-written by the finalisation item).
struct BState {
    int32_t status;        // BS_*
    int32_t have_prev;
    int64_t step;          // steps completed since admission
    double scale;          // pending renormalisation factor
    double norm;           // dV sum |psi|^2 after the last step (before renormalisation)
    double mu_prev;
    double obs[12];        // norm, mu, E, K, P, I, <x>, <y>, <z>, <x^2>, <y^2>, <z^2> at the last observation
    int64_t obs_step;
};

struct BItem {
    uint16_t slot;
    uint8_t pass;
    uint8_t pad_;
    int32_t tile;
};

// Counters and the work-list header.
struct BCtl {
    int32_t ticket;
    int32_t exited;
    int32_t total_items;
    int32_t error;         // bit 0: a bounded wait gave up; bit 1: a solo line had no register-resident form;
                           // bit 2: an item's form was not in the launched kernel form
    int32_t max_slots;
    int32_t solo_min;      // steps a solo item takes before it may stop early
    int32_t reg_epoch;     // persistent launches completed since the work list was uploaded
    int32_t pad_[9];
};

struct BatchArgs {
    BCtl *ctl;
    int32_t *done;         // [max_slots][4] tiles completed per sweep / observation pass
    const BInst *inst;
    BState *state;
    const BItem *items;
    int32_t spin_limit;
};

hipError_t launch_batch_step(const BatchArgs &a, bool big, bool full, int grid, size_t lds, hipStream_t st);
hipError_t launch_batch_solo(const BatchArgs &a, bool big, int grid, size_t lds, hipStream_t st, int steps,
                             int target);
hipError_t batch_step_occupancy(bool big, size_t lds, int *blocks_per_cu);
hipError_t launch_batch_scale(int elem, void *psi, int64_t npts, double *scale, hipStream_t st);

}  // namespace sscn
