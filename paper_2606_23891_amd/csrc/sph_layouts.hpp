// Particle layouts (paper Sec. 3.1) as compile-time descriptor tables.
//
// A layout is a list of substructs; a substruct is a list of members placed
// in order at natural alignment, each record padded to 8 bytes.  SoA is one
// array per scalar component (the 40-byte cold block stays one element).
// Kernels are instantiated per layout, so every field access below folds to a
// constant substruct index, record stride and byte offset (the getter/setter
// mapping of Algorithm 1, resolved at compile time).
//
// A layout may hold the position x more than once (the data replication of
// Sec. 5: a copy in every substruct a loop reads).  The first copy in member
// order is the primary one, which every read takes; every write of x (store
// setters, drift, layout conversion) writes all copies.
#pragma once
#include <cstddef>
#include <cstdint>

namespace sph {

enum Field : int {
    FX, FV, FA, FMASS, FH, FU, FUDT, FRHO, FRHODH, FWCOUNT, FDIV, FROT, FLAP, FVSIG,
    FAV, FAD, FTBIN, FID, FCOLD, NFIELD
};
constexpr int kNComp[NFIELD] = {3, 3, 3, 1, 1, 1, 1, 1, 1, 1, 1, 3, 1, 1, 1, 1, 1, 1, 5};
constexpr int kCompBytes[NFIELD] = {8, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 1, 8, 8};

constexpr int kMaxSub = 32;
constexpr int kNLayouts = 10;
constexpr int kSoA = 8;
constexpr int kMaxXRep = 3;  // copies of x beyond the primary one

struct LayoutDesc {
    int nsub;
    int sub_bytes[kMaxSub];
    int sub[NFIELD][5];
    int off[NFIELD][5];
    int nxrep;                 // replicas of x
    int xrep_sub[kMaxXRep];    // substruct of replica r
    int xrep_off[kMaxXRep];    // byte offset of its component 0 (components 8 bytes apart)
};

constexpr int kNext = -2, kEnd = -1;

// Member lists.  Usage order of the AoS record follows the paper's remark that
// members sit in the order the code uses them.
constexpr int kListAoS[] = {FX, FV, FA, FMASS, FH, FU, FUDT, FRHO, FRHODH, FWCOUNT, FDIV, FROT,
                            FLAP, FVSIG, FAV, FAD, FTBIN, FID, FCOLD, kEnd};
// the AoS members in a fixed shuffled order (numpy PCG64, seed 0, permutation of 19)
constexpr int kListRandom[] = {FA, FDIV, FMASS, FAV, FX, FLAP, FH, FCOLD, FRHO, FU, FID, FTBIN,
                               FRHODH, FROT, FUDT, FVSIG, FWCOUNT, FV, FAD, kEnd};
// pack-gradient: {gradient pack set} {force-only inputs} {outputs} {cold}
constexpr int kListGrad[] = {FX, FV, FMASS, FH, FU, FRHO, kNext,
                             FRHODH, FDIV, FROT, FAV, FAD, kNext,
                             FA, FUDT, FWCOUNT, FLAP, FVSIG, kNext,
                             FTBIN, FID, FCOLD, kEnd};
// pack-force: {force pack set} {outputs} {cold}
constexpr int kListForce[] = {FX, FV, FMASS, FH, FU, FRHO, FRHODH, FDIV, FROT, FAV, FAD, kNext,
                              FA, FUDT, FWCOUNT, FLAP, FVSIG, kNext,
                              FTBIN, FID, FCOLD, kEnd};
// pack-shared: {x m h used by every loop} {v u rho} {force-only} {outputs} {cold}
constexpr int kListShared[] = {FX, FMASS, FH, kNext,
                               FV, FU, FRHO, kNext,
                               FRHODH, FDIV, FROT, FAV, FAD, kNext,
                               FA, FUDT, FWCOUNT, FLAP, FVSIG, kNext,
                               FTBIN, FID, FCOLD, kEnd};
// pack-shared with replicated positions: x in every substruct a loop packs from
constexpr int kListSharedRepl[] = {FX, FMASS, FH, kNext,
                                   FX, FV, FU, FRHO, kNext,
                                   FX, FRHODH, FDIV, FROT, FAV, FAD, kNext,
                                   FA, FUDT, FWCOUNT, FLAP, FVSIG, kNext,
                                   FTBIN, FID, FCOLD, kEnd};
// type-split variants: double / float / integer / opaque parts of each substruct
constexpr int kListGradT[] = {FX, kNext, FV, FMASS, FH, FU, FRHO, kNext,
                              FRHODH, FDIV, FROT, FAV, FAD, kNext,
                              FA, FUDT, FWCOUNT, FLAP, FVSIG, kNext,
                              FTBIN, FID, kNext, FCOLD, kEnd};
constexpr int kListForceT[] = {FX, kNext, FV, FMASS, FH, FU, FRHO, FRHODH, FDIV, FROT, FAV, FAD, kNext,
                               FA, FUDT, FWCOUNT, FLAP, FVSIG, kNext,
                               FTBIN, FID, kNext, FCOLD, kEnd};
constexpr int kListSharedT[] = {FX, kNext, FMASS, FH, kNext,
                                FV, FU, FRHO, kNext,
                                FRHODH, FDIV, FROT, FAV, FAD, kNext,
                                FA, FUDT, FWCOUNT, FLAP, FVSIG, kNext,
                                FTBIN, FID, kNext, FCOLD, kEnd};

constexpr LayoutDesc build_list(const int *list)
{
    LayoutDesc d{};
    int s = 0, off = 0;
    bool have_x = false;
    for (int k = 0;; ++k) {
        const int f = list[k];
        if (f == kNext || f == kEnd) {
            d.sub_bytes[s] = (off + 7) / 8 * 8;
            ++s;
            off = 0;
            if (f == kEnd) break;
            continue;
        }
        const int align = kCompBytes[f] < 8 ? kCompBytes[f] : 8;
        off = (off + align - 1) / align * align;
        if (f == FX && have_x) {
            d.xrep_sub[d.nxrep] = s;
            d.xrep_off[d.nxrep] = off;
            ++d.nxrep;
        } else {
            for (int c = 0; c < kNComp[f]; ++c) {
                d.sub[f][c] = s;
                d.off[f][c] = off + c * kCompBytes[f];
            }
            if (f == FX) have_x = true;
        }
        off += kNComp[f] * kCompBytes[f];
    }
    d.nsub = s;
    return d;
}

// is component (f, c) stored in substruct s (as the primary copy or a replica
// of x), and at which byte offset of the record
constexpr bool has_member(const LayoutDesc &d, int f, int c, int s)
{
    if (d.sub[f][c] == s) return true;
    if (f == FX)
        for (int r = 0; r < d.nxrep; ++r)
            if (d.xrep_sub[r] == s) return true;
    return false;
}
constexpr int member_off(const LayoutDesc &d, int f, int c, int s)
{
    if (d.sub[f][c] == s) return d.off[f][c];
    for (int r = 0; r < d.nxrep; ++r)
        if (d.xrep_sub[r] == s) return d.xrep_off[r] + 8 * c;
    return -1;
}

constexpr LayoutDesc build_soa()
{
    LayoutDesc d{};
    int s = 0;
    for (int f = 0; f < NFIELD; ++f) {
        if (f == FCOLD) {
            for (int c = 0; c < 5; ++c) {
                d.sub[f][c] = s;
                d.off[f][c] = 8 * c;
            }
            d.sub_bytes[s++] = 40;
            continue;
        }
        for (int c = 0; c < kNComp[f]; ++c) {
            d.sub[f][c] = s;
            d.off[f][c] = 0;
            d.sub_bytes[s++] = kCompBytes[f];
        }
    }
    d.nsub = s;
    return d;
}

constexpr LayoutDesc kLayouts[kNLayouts] = {
    build_list(kListAoS),   build_list(kListRandom), build_list(kListGrad),
    build_list(kListForce), build_list(kListShared), build_list(kListGradT),
    build_list(kListForceT), build_list(kListSharedT), build_soa(), build_list(kListSharedRepl)};

static_assert(kLayouts[0].nsub == 1 && kLayouts[0].sub_bytes[0] == 160, "AoS record is 160 bytes");
static_assert(kLayouts[1].sub_bytes[0] == 160, "shuffled AoS record");
static_assert(kLayouts[kSoA].nsub == 27, "SoA arrays");
static_assert(kLayouts[9].nxrep == 2 && kLayouts[9].sub_bytes[1] == 48 && kLayouts[9].sub_bytes[2] == 56,
              "replicated positions: x in three substructs");

}  // namespace sph
