// Host emulation of the tiled kernels, lane by lane, for tests and layout
// checks.  It runs the plan the device path would run, with the same tables
// and the same slot / lane / iteration arithmetic as TileCtx in kernels.hip,
// and counts what the paper's arguments are about: global accesses per wave
// (coalescing, Section 4.1), LDS bank conflicts (Section 4.2) and whether
// every LDS slot of a tile is written once and read once.  The device entry
// points never call this.
#include <cstring>
#include <set>
#include <vector>

#include "runtime.hpp"

namespace bmmc {

namespace {

uint32_t lin(const uint32_t* tab, int base, int nbits, uint32_t v) {
    uint32_t r = 0;
    for (int k = 0; k < nbits; k++)
        if ((v >> k) & 1u) r ^= tab[base + k];
    return r;
}

// Extra cycles of one wave LDS access: lanes are served in groups of
// nb*4/w; in a group, a bank holding k distinct dwords costs k cycles.
int64_t lds_extra(const std::vector<int64_t>& slot_of_lane, int w, int nb) {
    if (w < 4) return 0;
    int g = nb * 4 / w;
    if (g > 64) g = 64;
    const int dw = w / 4;
    int64_t extra = 0;
    for (int base = 0; base < 64; base += g) {
        std::vector<std::set<int64_t>> bank(nb);
        bool any = false;
        for (int l = base; l < base + g; l++) {
            const int64_t s = slot_of_lane[l];
            if (s < 0) continue;
            any = true;
            for (int q = 0; q < dw; q++) {
                const int64_t a = s * dw + q;
                bank[a % nb].insert(a);
            }
        }
        if (!any) continue;
        size_t worst = 0;
        for (auto& b : bank) worst = b.size() > worst ? b.size() : worst;
        extra += (int64_t)worst - 1;
    }
    return extra;
}

int64_t lines_of(const std::vector<int64_t>& byte_of_lane, int* active) {
    std::set<int64_t> lines;
    int act = 0;
    for (int64_t b : byte_of_lane) {
        if (b < 0) continue;
        act++;
        lines.insert(b / 128);
        lines.insert((b + 15) / 128);
    }
    *active = act;
    return (int64_t)lines.size();
}

void emulate_pass(const PassTables& P, const KernelShape& ks, int w, const uint8_t* src, uint8_t* dst,
                  bmmc_emu_stats_t* st) {
    const int VEC = 16 / w, LV = ks.lv(), LT = ks.lt(), LI = ks.li(), NT = ks.nt, IT = ks.iters;
    const int D = LV + LT + LI;
    const uint32_t ntiles = 1u << P.ntb;
    const uint32_t vlim = 1u << (P.d - LV);
    std::vector<uint8_t> lds((size_t)w << D);
    std::vector<int> wr((size_t)1 << D), rd((size_t)1 << D);
    std::vector<uint32_t> xt(NT), ft(NT), yt(NT), gt(NT);
    for (int tid = 0; tid < NT; tid++) {
        xt[tid] = lin(P.X, LV, LT, tid);
        ft[tid] = lin(P.F, LV, LT, tid);
        yt[tid] = lin(P.Y, LV, LT, tid);
        gt[tid] = lin(P.G, LV, LT, tid);
    }
    std::vector<int64_t> lane_bytes(64), lane_slot(64);
    uint32_t class0 = 0;  // 4 KiB-block class (block index mod 8) written by tile 0
    for (uint32_t tile = 0; tile < ntiles; tile++) {
        st->tiles++;
        uint32_t classes = 0;  // bit k: the tile writes a block of class k
        uint32_t r = 0, yb = P.c_hi, gx = P.c_lds;
        for (uint32_t j = 0; j < P.ntb; j++)
            if ((tile >> j) & 1u) {
                r ^= P.tb[j][0];
                yb ^= P.tb[j][1];
                gx ^= P.tb[j][2];
            }
        std::fill(wr.begin(), wr.end(), 0);
        std::fill(rd.begin(), rd.end(), 0);
        // read phase
        for (int it = 0; it < IT; it++) {
            for (int wave = 0; wave < NT / 64; wave++) {
                int active;
                for (int l = 0; l < 64; l++) {
                    const uint32_t tid = wave * 64 + l;
                    lane_bytes[l] = ((uint32_t)(it * NT) + tid < vlim)
                                        ? (int64_t)(r ^ xt[tid] ^ lin(P.X, LV + LT, LI, it)) * w
                                        : -1;
                }
                const int64_t lines = lines_of(lane_bytes, &active);
                if (active) {
                    st->read_instr++;
                    st->read_lines += lines;
                    st->read_lines_min += (active * 16 + 127) / 128;
                }
                for (int e = 0; e < VEC; e++) {
                    for (int l = 0; l < 64; l++) {
                        const uint32_t tid = wave * 64 + l;
                        if (lane_bytes[l] < 0) {
                            lane_slot[l] = -1;
                            continue;
                        }
                        const uint32_t slot = ft[tid] ^ lin(P.F, LV + LT, LI, it) ^ lin(P.F, 0, LV, e);
                        lane_slot[l] = slot;
                        std::memcpy(&lds[(size_t)slot * w], src + lane_bytes[l] + (int64_t)e * w, w);
                        wr[slot]++;
                    }
                    if (active) {
                        st->lds_instr++;
                        st->lds_conflicts32 += lds_extra(lane_slot, w, 32);
                        st->lds_conflicts64 += lds_extra(lane_slot, w, 64);
                    }
                }
            }
        }
        // write phase
        for (int it = 0; it < IT; it++) {
            for (int wave = 0; wave < NT / 64; wave++) {
                int active = 0;
                for (int l = 0; l < 64; l++) {
                    const uint32_t tid = wave * 64 + l;
                    lane_bytes[l] = ((uint32_t)(it * NT) + tid < vlim)
                                        ? (int64_t)(yb ^ yt[tid] ^ lin(P.Y, LV + LT, LI, it)) * w
                                        : -1;
                }
                for (int e = 0; e < VEC; e++) {
                    for (int l = 0; l < 64; l++) {
                        const uint32_t tid = wave * 64 + l;
                        if (lane_bytes[l] < 0) {
                            lane_slot[l] = -1;
                            continue;
                        }
                        const uint32_t slot = gt[tid] ^ gx ^ lin(P.G, LV + LT, LI, it) ^ lin(P.G, 0, LV, e);
                        lane_slot[l] = slot;
                        std::memcpy(dst + lane_bytes[l] + (int64_t)e * w, &lds[(size_t)slot * w], w);
                        rd[slot]++;
                    }
                    int act2 = 0;
                    for (int l = 0; l < 64; l++) act2 += lane_slot[l] >= 0;
                    if (act2) {
                        st->lds_instr++;
                        st->lds_conflicts32 += lds_extra(lane_slot, w, 32);
                        st->lds_conflicts64 += lds_extra(lane_slot, w, 64);
                    }
                }
                for (int l = 0; l < 64; l++)
                    if (lane_bytes[l] >= 0) classes |= 1u << ((lane_bytes[l] >> 12) & 7);
                const int64_t lines = lines_of(lane_bytes, &active);
                if (active) {
                    st->write_instr++;
                    st->write_lines += lines;
                    st->write_lines_min += (active * 16 + 127) / 128;
                }
            }
        }
        if (tile == 0 && classes) class0 = (uint32_t)__builtin_ctz(classes);
        if (classes == 1u << ((tile ^ class0) & 7u)) st->dealt_write_tiles++;
        const uint32_t valid_slots = vlim * VEC;
        for (uint32_t s = 0; s < ((uint32_t)1 << D); s++) {
            const bool valid = s < valid_slots;
            if (valid && (wr[s] != 1 || rd[s] != 1)) st->lds_slot_errors++;
            if (!valid && (wr[s] != 0 || rd[s] != 0)) st->lds_slot_errors++;
        }
    }
}

}  // namespace
}  // namespace bmmc

using namespace bmmc;

extern "C" int bmmc_emulate(const void* in, void* out, int n, const uint64_t* A_rows, uint64_t c,
                            int elem_bytes, const bmmc_options_t* opts, bmmc_emu_stats_t* stats) {
    if (!in || !out) return set_error(BMMC_ERR_ARG, "in/out must not be NULL");
    if (n < 0 || n > 30) return set_error(BMMC_ERR_RANGE, "emulation supports n <= 30");
    const bmmc_options_t eff = effective_options(nullptr, n, elem_bytes, opts);
    PlanOptions po = plan_options(&eff, elem_bytes);
    Plan p;
    int st = make_plan(A_rows, c, n, elem_bytes, po, &p);
    if (st != BMMC_OK) return set_error(st, "planning failed: %s", bmmc_strerror(st));
    bmmc_emu_stats_t local;
    std::memset(&local, 0, sizeof(local));
    const size_t bytes = ((size_t)1 << n) * (size_t)elem_bytes;
    const uint8_t* src = (const uint8_t*)in;
    uint8_t* dst = (uint8_t*)out;
    if (p.npass == 0) {
        std::memcpy(dst, src, bytes);
    } else if (p.naive) {
        for (uint64_t x = 0; x < ((uint64_t)1 << n); x++) {
            const uint64_t y = p.A.apply(x) ^ p.c;
            std::memcpy(dst + y * elem_bytes, src + x * elem_bytes, elem_bytes);
        }
    } else {
        std::vector<uint8_t> mid(p.npass == 2 ? bytes : 0);
        for (int k = 0; k < p.npass; k++) {
            const uint8_t* s = (k == 0) ? src : mid.data();
            uint8_t* d = (k == p.npass - 1) ? dst : mid.data();
            emulate_pass(p.pass[k].tab, p.shape, elem_bytes, s, d, &local);
        }
    }
    if (stats) *stats = local;
    return BMMC_OK;
}
