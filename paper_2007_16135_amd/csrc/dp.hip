// dp.hip -- the strip sweep run on the sibling recurrences (DTW, edit
// distance, the indel distance that gives the LCS length), as tiles with FP64
// accumulators.  Section "Generalized Dynamic Programming Extensions" of the
// paper points out that such programs need only the cells above, to the left
// and up-left, so the band sweep carries over unchanged; only the cell update
// differs (lane_row_sibling in twed_device.h).
#include "wavefront_impl.h"

#include <type_traits>

namespace twed {

namespace {

// Strip widths and group sizes compiled for the sibling recurrences.
template <int DIMT, int K>
constexpr bool kDpCompiled = (K == 1 || K == 2 || K == 8) && kStripCompiled<DIMT, K>;

template <int REC, int DIMT>
constexpr bool kDpDim = REC == kRecDtw || DIMT == 1;

template <typename CT, typename AT, int DIMT, int PM, int K, int G, int REC>
hipError_t launch_dp_kg(const WavefrontArgs &a, const TileIO<AT> &io, const CostParams &cp, hipStream_t st)
{
    hipLaunchKernelGGL((wavefront_kernel<CT, AT, DIMT, PM, K, G, false, true, REC>), dim3(a.grid), dim3(kWave * G), 0,
                       st, (const CT *)a.rowsA, (const CT *)a.rowsB, (int)a.nA, (int)a.nB, CostArgs<CT>::make(cp),
                       (Pair2<AT> *)a.bnd, a.flags, a.ticket, a.ticket + 1, (int)a.nStrips, (const CT *)a.beta,
                       (AT *)a.out, nullptr, a.sub_shift, io);
    return hipGetLastError();
}

template <typename Fn>
hipError_t by_rec(int rec, Fn &&fn)
{
    switch (rec) {
    case kRecDtw: return fn.template operator()<kRecDtw>();
    case kRecEdit: return fn.template operator()<kRecEdit>();
    case kRecIndel: return fn.template operator()<kRecIndel>();
    default: return hipErrorInvalidValue;
    }
}

// Calls fn.template operator()<CT, AT, DIMT, PM, K, G, REC>() for a compiled
// configuration, else returns hipErrorInvalidValue.
template <typename Fn>
hipError_t by_config(int rec, Prec prec, const CostParams &cp, int K, int G, Fn &&fn)
{
    if (prec != kF64 && prec != kF32Acc64) return hipErrorInvalidValue;
    return by_rec(rec, [&]<int REC>() -> hipError_t {
        return by_prec(prec, cp.dimt, cp.pm, [&]<typename CT, typename AT, int DIMT, int PM>() -> hipError_t {
            if constexpr (!std::is_same_v<AT, double> || !kDpDim<REC, DIMT>) {
                return hipErrorInvalidValue;
            } else {
                auto withK = [&]<int KK>() -> hipError_t {
                    if constexpr (!kDpCompiled<DIMT, KK>) {
                        return hipErrorInvalidValue;
                    } else {
                        switch (G) {
                        case 1: return fn.template operator()<CT, AT, DIMT, PM, KK, 1, REC>();
                        case 8: return fn.template operator()<CT, AT, DIMT, PM, KK, 8, REC>();
                        default: return hipErrorInvalidValue;
                        }
                    }
                };
                switch (K) {
                case 1: return withK.template operator()<1>();
                case 2: return withK.template operator()<2>();
                case 8: return withK.template operator()<8>();
                default: return hipErrorInvalidValue;
                }
            }
        });
    });
}

}  // namespace

hipError_t launch_dp(int rec, Prec prec, const CostParams &cp, int K, const WavefrontArgs &a, const TileArgs &t,
                     hipStream_t st)
{
    if (t.dirs) return launch_rec_dirs(rec, prec, cp, K, a, t, st);
    hipError_t e = by_config(rec, prec, cp, K, a.group,
                             [&]<typename CT, typename AT, int DIMT, int PM, int KK, int G, int REC>() -> hipError_t {
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
                                 return launch_dp_kg<CT, AT, DIMT, PM, KK, G, REC>(a, io, cp, st);
                             });
    if (e != hipSuccess) return e;
    return launch_tile_edges(a.nA, a.nB, t, st);
}

size_t dp_scratch_bytes(int rec, Prec prec, const CostParams &cp, int K, int G)
{
    size_t bytes = (size_t)-1;
    (void)by_config(rec, prec, cp, K, G, [&]<typename CT, typename AT, int DIMT, int PM, int KK, int GG, int REC>() {
        bytes = scratch_kg<CT, AT, DIMT, PM, KK, GG, true, REC>();
        return hipSuccess;
    });
    return bytes;
}

int dp_max_workers(int rec, Prec prec, const CostParams &cp, int K, int G)
{
    int per_cu = 0;
    (void)by_config(rec, prec, cp, K, G, [&]<typename CT, typename AT, int DIMT, int PM, int KK, int GG, int REC>() {
        per_cu = occupancy_kg<CT, AT, DIMT, PM, KK, GG, true, REC>();
        return hipSuccess;
    });
    if (per_cu <= 0) return 0;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return per_cu * cus;
}

}  // namespace twed
