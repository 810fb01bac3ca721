// Per-worker chunk and LDS-slot planner (part of the layout step, section 3.1: the data
// of a worker is fixed once the rows are partitioned, so its whole schedule within an
// epoch is known in advance).
//
// Worker q processes its ratings in ring order (sub-step, item, row).  The planner cuts
// that sequence into chunks of at most 64 ratings inside one block and manages the S
// LDS slots of the worker like a register allocator with a known future:
//   * an item is loaded at the start of its visit (its run of ratings in the block) and
//     released after the chunk holding the visit's last rating;
//   * a row stays in its slot until a load needs the slot.  The victim is chosen among
//     slots the current chunk does not use, preferring (0) free slots released at least
//     `look` chunks ago, (1) rows unused for `look` chunks with the farthest next use
//     (Belady), then (2) recently freed slots and (3) recently used rows.  A load into a
//     slot whose previous vector was used by chunk c' can only be staged once the compute
//     wave has finished chunk c'; preferring old victims lets the memory wave stage a
//     chunk while the chunks before it are computed.
// Rows left in LDS at the end of the epoch are listed with the last chunk (written back
// there), so every epoch starts with empty slots.
//
// The function is written once for the host and the device: the layout kernel runs it
// with one thread per worker, first counting (kFill = false) and then writing.
#pragma once

#include <stdint.h>

#include "nomad_internal.h"

namespace nomad {

struct PlanIn {
    const int32_t *srow, *scol;
    const float *sval;
    const uint32_t *blk;    // per rating: block key q * p + s (changes at block boundaries)
    const uint32_t *vinfo;  // per rating: v | nvis << 16 of the visit it belongs to
    int32_t slots, cap, look;
    int32_t *nxt;           // scratch per rating: next position of the same row (-1: none)
    int32_t *rowmap;        // scratch per row, -1 on entry and on return; during the forward
                            // pass: LDS slot, -1 (not in LDS) or -2 - c (evicted by chunk c)
};

struct PlanOut {
    ChunkRec *chunks;
    EvRec *events;
    RatingRec *ratings;
    int64_t ck0, ev0;       // first chunk / event record of the worker
};

struct PlanCount {
    int64_t chunks, events, loads;
    int32_t status;         // 0 ok, 1 slots too few for one rating
};

template <bool kFill>
__host__ __device__ PlanCount plan_worker(const PlanIn &in, int64_t e0, int64_t e1, const PlanOut &out) {
    PlanCount res{0, 0, 0, 0};
    if (e1 <= e0) return res;
    const int32_t S = in.slots;
    constexpr int32_t kNone = 0x7fffffff;

    // Next use of each rating's row (position relative to e0), by a backward pass.
    for (int64_t e = e1 - 1; e >= e0; --e) {
        const int32_t i = in.srow[e];
        in.nxt[e] = in.rowmap[i];
        in.rowmap[i] = (int32_t)(e - e0);
    }
    for (int64_t e = e0; e < e1; ++e) in.rowmap[in.srow[e]] = -1;

    int32_t occ[kMaxSlots];    // row or item id held, -1 = free
    uint8_t isitem[kMaxSlots];
    int32_t last[kMaxSlots];   // last chunk using the occupant (or that released the slot)
    int32_t nextu[kMaxSlots];  // rows: next position using the row
    for (int32_t s = 0; s < S; ++s) {
        occ[s] = -1;
        isitem[s] = 0;
        last[s] = -1;
        nextu[s] = kNone;
    }
    EvRec ld[kMaxEventsPerChunk], rl[kMaxEventsPerChunk];

    int32_t c = 0, nrat = 0, nload = 0, nrel = 0, need = 0;
    int64_t rat0 = e0, ev_pos = 0;
    int32_t cur_item = -1, cur_slot = -1;
    uint32_t cur_vis = 0, cur_blk = 0xffffffffu;
    bool item_in_c = false;

    auto emit_chunk = [&](int32_t nflush) {
        if (kFill) {
            ChunkRec r;
            r.rat = rat0;
            r.ev = out.ev0 + ev_pos;
            r.nrat = (uint16_t)nrat;
            r.nload = (uint16_t)nload;
            r.nrel = (uint16_t)nrel;
            r.nflush = (uint16_t)nflush;
            r.need_done = need;
            r.flags = 0;
            out.chunks[out.ck0 + c] = r;
            for (int32_t x = 0; x < nload; ++x) out.events[out.ev0 + ev_pos + x] = ld[x];
            for (int32_t x = 0; x < nrel; ++x) out.events[out.ev0 + ev_pos + nload + x] = rl[x];
        }
        ev_pos += nload + nrel;
        res.loads += nload;
    };
    auto close_chunk = [&](int64_t next_rat) {
        emit_chunk(0);
        ++c;
        nrat = nload = nrel = need = 0;
        rat0 = next_rat;
        item_in_c = false;
    };
    auto end_item_run = [&]() {
        EvRec r;
        r.id = cur_item;
        r.sk = (uint32_t)cur_slot | (kEvRelease << 8);
        r.evict = -1;
        r.vis = cur_vis;
        rl[nrel++] = r;
        occ[cur_slot] = -1;
        isitem[cur_slot] = 0;
        last[cur_slot] = c;
        cur_item = -1;
        cur_slot = -1;
        item_in_c = false;
    };
    // Slot for a vector loaded by chunk c, or -1 if every slot is taken by chunk c.
    auto find_slot = [&]() -> int32_t {
        int32_t best = -1, best_cls = 4, best_last = 0, best_next = 0;
        for (int32_t s = 0; s < S; ++s) {
            if (last[s] >= c || s == cur_slot) continue;
            const bool old = last[s] <= c - 1 - in.look;
            const int32_t cls = occ[s] < 0 ? (old ? 0 : 2) : (old ? 1 : 3);
            bool better = cls < best_cls;
            if (cls == best_cls) {
                if (cls == 1 || cls == 3)
                    better = nextu[s] > best_next || (nextu[s] == best_next && last[s] < best_last);
                else
                    better = last[s] < best_last;
            }
            if (better) {
                best = s;
                best_cls = cls;
                best_last = last[s];
                best_next = nextu[s];
            }
        }
        return best;
    };
    // Load a vector into a free or evicted slot for chunk c.
    auto take_slot = [&](int32_t s, int32_t id, bool item, uint32_t vis) {
        EvRec r;
        r.id = id;
        r.sk = (uint32_t)s | ((item ? kEvLoadItem : kEvLoadRow) << 8);
        r.evict = -1;
        r.vis = vis;
        if (occ[s] >= 0) {  // a row: written back first
            r.evict = occ[s];
            in.rowmap[occ[s]] = -2 - c;
        }
        const int32_t nd = last[s] + 1;
        if (nd > need) need = nd;
        ld[nload++] = r;
        occ[s] = id;
        isitem[s] = item ? 1 : 0;
        last[s] = c;
        nextu[s] = kNone;
    };

    for (int64_t e = e0; e < e1; ++e) {
        const int32_t i = in.srow[e], j = in.scol[e];
        const uint32_t b = in.blk[e];
        const bool new_blk = b != cur_blk;
        const bool new_item = new_blk || j != cur_item;
        if (new_item && cur_item >= 0) end_item_run();
        if (new_blk && nrat > 0) close_chunk(e);
        cur_blk = b;
        for (int attempt = 0;; ++attempt) {
            // A row evicted by the open chunk is not loaded again by it: the memory wave
            // may read a chunk's rows before it writes back the rows that chunk evicts.
            if (in.rowmap[i] == -2 - c) {
                close_chunk(e);
                continue;
            }
            const int32_t rs = in.rowmap[i] >= 0 ? in.rowmap[i] : -1;
            const int32_t need_loads = (rs < 0 ? 1 : 0) + (cur_item < 0 ? 1 : 0);
            const int32_t reserve = item_in_c ? 0 : 1;  // release event of this rating's item
            const int32_t events = nload + nrel + (item_in_c ? 1 : 0);
            if (nrat > 0 && (nrat == kMaxRatingsPerChunk || nload + need_loads > in.cap ||
                             events + need_loads + reserve > kMaxEventsPerChunk)) {
                close_chunk(e);
                continue;
            }
            if (rs >= 0) last[rs] = c;  // this rating's row must not be the item's victim
            if (cur_item < 0) {
                const int32_t s = find_slot();
                if (s < 0) {
                    if (nrat == 0 && nload == 0) { res.status = 1; return res; }
                    close_chunk(e);
                    continue;
                }
                take_slot(s, j, true, in.vinfo[e]);
                cur_item = j;
                cur_slot = s;
                cur_vis = in.vinfo[e];
            }
            if (rs < 0) {
                if (nload + 1 > in.cap) {  // the item took the last load of the chunk
                    close_chunk(e);
                    continue;
                }
                const int32_t s = find_slot();
                if (s < 0) {
                    if (nrat == 0 && nload <= 1 && attempt > 1) { res.status = 1; return res; }
                    close_chunk(e);
                    continue;
                }
                take_slot(s, i, false, 0u);
                in.rowmap[i] = s;
            }
            break;
        }
        const int32_t rs = in.rowmap[i];
        last[rs] = c;
        nextu[rs] = in.nxt[e] < 0 ? kNone : in.nxt[e];
        last[cur_slot] = c;
        item_in_c = true;
        if (kFill) {
            RatingRec rr;
            rr.slots = (uint32_t)rs | ((uint32_t)cur_slot << 8);
            rr.r = in.sval[e];
            out.ratings[e] = rr;
        }
        ++nrat;
    }
    if (cur_item >= 0) end_item_run();
    // Last chunk: rows still in LDS are written back after it.
    int32_t nflush = 0;
    for (int32_t s = 0; s < S; ++s) {
        if (occ[s] < 0 || isitem[s]) continue;
        if (kFill) {
            EvRec r;
            r.id = occ[s];
            r.sk = (uint32_t)s | (kEvFlush << 8);
            r.evict = -1;
            r.vis = 0;
            out.events[out.ev0 + ev_pos + nload + nrel + nflush] = r;
        }
        in.rowmap[occ[s]] = -1;
        ++nflush;
    }
    for (int64_t e = e0; e < e1; ++e) in.rowmap[in.srow[e]] = -1;
    emit_chunk(nflush);
    ev_pos += nflush;
    ++c;
    res.chunks = c;
    res.events = ev_pos;
    return res;
}

}  // namespace nomad
