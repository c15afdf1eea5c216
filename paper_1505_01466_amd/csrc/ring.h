// Device-visible request ring of the persistent serving mode (internal to
// the library: shared by decoder.hip, which holds the kernel, and
// server.cpp, which fills the ring).
//
// The host publishes requests into memory both sides see coherently
// (pinned, coherent host memory): a record per published frame (its rows,
// its request's slot, ticket, plan and frame count; frames are numbered
// globally in publication order) and the count of published frames.  A
// persistent kernel's workgroups take frames one at a time by ticket (see
// Dev), decode them with their request's plan, and count them per slot (and
// all of them in Dev::done); the last frame of a
// request writes the request's ticket to its completion word.  A workgroup
// leaves when the host raises `stop` or after `idle_us` microseconds without
// a frame to claim, so every launch ends on its own; the host relaunches
// when requests are held and no launch is running, and a new launch
// continues from the device counter.
#ifndef PSCL_RING_H
#define PSCL_RING_H

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include "pscl.h"

namespace pscl_ring {

struct Rec {  // one published frame (64 bytes, read by one wavefront load)
    const void* llr;  // the frame's LLR row
    uint8_t* u_hat;   // its output row
    uint8_t* crc_ok;  // its flag (or NULL)
    void* pm;         // its metric (or NULL)
    uint64_t ticket;  // of its request
    uint32_t slot;    // of its request
    int32_t plan;
    int64_t F;        // frames of its request
    int64_t pad;
};
static_assert(sizeof(Rec) == 64, "a frame record is eight 8-byte words");

struct Ctl {
    uint64_t published;  // frames published so far
    uint32_t stop;       // 1: every workgroup leaves at its next claim
    uint32_t active;     // workgroups per CU that take frames (by launch rank;
                         // 0: as many as the frames outstanding call for)
};

// Device-side state.  A free workgroup takes a ticket, the number of the
// global frame it will decode (first from the frames the previous launch
// left unclaimed, then a new number from `next`, one atomic add: no
// retries), and waits until that frame is published.  Idle workgroups read
// host memory one at a time (whoever takes the lease copies the published
// count and the stop flag into `published` / `stop`); the others poll
// these copies.  A workgroup that leaves holding a ticket of an unpublished
// frame records it in the orphan list of its launch's parity (at most one
// per workgroup); the next launch takes those tickets first.  The host
// clears orphan_n[p] and orphan_take[1 - p] before a launch of parity p.
// Each group of words that different workgroups poll or update sits in a
// cache line of its own.
struct Dev {
    alignas(128) unsigned long long next;  // next new ticket
    alignas(128) unsigned long long published;  // latest published count seen
    alignas(128) uint32_t lease;           // 1 while a workgroup reads host memory
    alignas(128) uint32_t stop;
    uint32_t active;                       // latest `active` seen
    alignas(128) unsigned long long done;  // frames finished so far (every launch)
    alignas(128) uint32_t orphan_n[2];     // tickets left by the launch of each parity
    uint32_t orphan_take[2];               // of those, taken by the next launch
};

struct Args {
    Ctl* ctl;                   // host-coherent
    const Rec* rec;             // host-coherent: global frame g at g & rec_mask
    uint64_t* done;             // host-coherent: ticket of the slot's finished request
    uint32_t* count;            // device: frames of the slot finished so far
    Dev* dev;                   // device
    unsigned long long* orphans;  // device: 2 x orphan_cap tickets
    uint32_t orphan_cap;        // at least the launch's workgroups
    uint32_t parity;            // of this launch
    uint32_t rec_mask;
    uint32_t idle_us;
    uint32_t wg_per_cu;  // resident workgroups per CU at most (0: as many as fit)
    uint32_t cus;        // compute units (set by launch)
    uint32_t* cu_rank;   // device, kCuSlots counters: workgroups started per CU
};

// Counters of workgroups per compute unit, indexed by the unit's hardware
// identity (XCC, shader engine, shader array, CU).
constexpr int kCuSlots = 2048;

// Launches the persistent serving kernel for the plans of group g (its
// concatenated schedules, plan table, first workspace, grid and LDS) on
// stream s.  Asynchronous.
pscl_status launch(pscl_group* g, const Args& a, hipStream_t s);

}  // namespace pscl_ring

#endif
