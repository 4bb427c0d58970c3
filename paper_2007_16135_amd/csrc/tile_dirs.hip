// tile_dirs.hip -- the tile sweep that also records the move into every cell
// (one byte per cell, for reading an alignment path back).  Kept apart from
// tile.hip: the recording code needs registers that the plain tile kernels
// then do not pay for.  Strips of one column per lane only (the blocks this
// sweeps are a few thousand columns wide).
#include "wavefront_impl.h"

#include <type_traits>

namespace twed {

namespace {

template <typename CT, typename AT, int DIMT, int PM, int G, int REC>
hipError_t launch_g(const WavefrontArgs &a, const TileIO<AT> &io, const CostParams &cp, hipStream_t st)
{
    hipLaunchKernelGGL((wavefront_kernel<CT, AT, DIMT, PM, 1, G, false, true, REC, true>), dim3(a.grid),
                       dim3(kWave * G), 0, st, (const CT *)a.rowsA, (const CT *)a.rowsB, (int)a.nA, (int)a.nB,
                       CostArgs<CT>::make(cp), (Pair2<AT> *)a.bnd, a.flags, a.ticket, a.ticket + 1, (int)a.nStrips,
                       (const CT *)a.beta, (AT *)a.out, nullptr, a.sub_shift, io);
    return hipGetLastError();
}

template <int REC, int DIMT>
constexpr bool kRecDim = REC == kRecTwed || REC == kRecDtw || DIMT == 1;

// fn.template operator()<CT, AT, DIMT, PM, G, REC>() for a compiled
// configuration (K = 1; G = 1, 4 or 8; FP64 accumulators).
template <typename Fn>
hipError_t by_config(int rec, Prec prec, const CostParams &cp, int G, Fn &&fn)
{
    if (prec != kF64 && prec != kF32Acc64) return hipErrorInvalidValue;
    auto with_rec = [&]<int REC>() -> hipError_t {
        return by_prec(prec, cp.dimt, cp.pm, [&]<typename CT, typename AT, int DIMT, int PM>() -> hipError_t {
            if constexpr (!std::is_same_v<AT, double> || !kRecDim<REC, DIMT>) {
                return hipErrorInvalidValue;
            } else {
                switch (G) {
                case 1: return fn.template operator()<CT, AT, DIMT, PM, 1, REC>();
                case 4: return fn.template operator()<CT, AT, DIMT, PM, 4, REC>();
                case 8: return fn.template operator()<CT, AT, DIMT, PM, 8, REC>();
                default: return hipErrorInvalidValue;
                }
            }
        });
    };
    switch (rec) {
    case kRecTwed: return with_rec.template operator()<kRecTwed>();
    case kRecDtw: return with_rec.template operator()<kRecDtw>();
    case kRecEdit: return with_rec.template operator()<kRecEdit>();
    case kRecIndel: return with_rec.template operator()<kRecIndel>();
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_rec_dirs(int rec, Prec prec, const CostParams &cp, int K, const WavefrontArgs &a, const TileArgs &t,
                           hipStream_t st)
{
    if (K != 1 || !t.dirs) return hipErrorInvalidValue;
    hipError_t e = by_config(rec, prec, cp, a.group, [&]<typename CT, typename AT, int DIMT, int PM, int G, int REC>() {
        TileIO<AT> io{};
        io.top = (const Pair2<AT> *)t.top;
        io.left = (const Pair2<AT> *)t.left;
        io.bottom = (Pair2<AT> *)t.bottom;
        io.right = (Pair2<AT> *)t.right;
        io.ckrow = (Pair2<AT> *)t.ckrow;
        io.ckcol = (Pair2<AT> *)t.ckcol;
        io.dummy = (Pair2<AT> *)t.dummy;
        io.dirs = t.dirs;
        io.ck_rows = t.ck_rows;
        io.ck_cols = t.ck_cols;
        return launch_g<CT, AT, DIMT, PM, G, REC>(a, io, cp, st);
    });
    if (e != hipSuccess) return e;
    return launch_tile_edges(a.nA, a.nB, t, st);
}

hipError_t launch_tile_dirs(Prec prec, const CostParams &cp, int K, const WavefrontArgs &a, const TileArgs &t,
                            hipStream_t st)
{
    return launch_rec_dirs(kRecTwed, prec, cp, K, a, t, st);
}

size_t rec_dirs_scratch_bytes(int rec, Prec prec, const CostParams &cp, int K, int G)
{
    size_t bytes = (size_t)-1;
    if (K != 1) return bytes;
    (void)by_config(rec, prec, cp, G, [&]<typename CT, typename AT, int DIMT, int PM, int GG, int REC>() {
        bytes = scratch_kg<CT, AT, DIMT, PM, 1, GG, true, REC, true>();
        return hipSuccess;
    });
    return bytes;
}

int rec_dirs_max_workers(int rec, Prec prec, const CostParams &cp, int K, int G)
{
    int per_cu = 0;
    if (K != 1) return 0;
    (void)by_config(rec, prec, cp, G, [&]<typename CT, typename AT, int DIMT, int PM, int GG, int REC>() {
        per_cu = occupancy_kg<CT, AT, DIMT, PM, 1, GG, true, REC, true>();
        return hipSuccess;
    });
    if (per_cu <= 0) return 0;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return per_cu * cus;
}

}  // namespace twed
