// wavefront.hip -- single-pair TWED sweep as a persistent pipeline of waves.
//
// The paper's section "Improved Time Warp Edit Distance" shows that cell
// (row, col) needs only its up, left and up-left neighbours, so the cells of
// one anti-diagonal (Eq. (1): diagonal = row + col, index = col) are
// independent and only three diagonals are ever live.  Its implementation
// (section "cuTWED Implementation Remarks") launches one grid per diagonal.
// Here the band is carried in registers instead:
//
//  * The columns 1..nB are cut into strips of 64*K.  One wave owns a strip;
//    lane l owns K consecutive columns and at step t works on row t - l, so
//    the wave's 64 lanes always hold a 64-cell segment of one anti-diagonal,
//    and the three live diagonals of that segment are the lane registers
//    (up, left and the match operand, see Lane in twed_device.h).
//  * The left and up-left operands of a lane's first column come from lane
//    l-1 through one DPP wave shift per step.
//  * Lane 0 of strip s takes them from the right-boundary column of strip
//    s-1 (DP and DP+e per row), one broadcast LDS read per step.  Lane 63
//    of strip s-1 writes that column to LDS as it produces it, one row per
//    step: into the ring the next wave of the workgroup reads, or into a
//    staging ring from which whole windows of rows go to one of two global
//    slots, published with a release flag; the consumer polls the flag and
//    acquires before copying the window into its own LDS.  Two slots
//    suffice: strip s+2 can only write row r after strip s+1 has published
//    row r, which it does after reading it.
//  * Waves take strips from an atomic ticket, so the wave that strip s waits
//    for has always started: no co-residency assumption, no deadlock.
//
// Memory stays O(nA + nB): packed inputs, two boundary columns, one flag per
// strip.  Every cell is evaluated once, in the operation order of the lane
// code, so the result does not depend on scheduling.
#include "wavefront_impl.h"

namespace twed {

template <typename CT, typename AT, int DIMT, int PM, int K, int G>
static hipError_t launch_kg(const WavefrontArgs &a, const CostParams &cp, hipStream_t st)
{
    if (a.dump) {
        // cell dumps are a validation aid: narrow strips, one wave per group
        if constexpr (K <= 2 && G == 1) {
            hipLaunchKernelGGL((wavefront_kernel<CT, AT, DIMT, PM, K, G, true, false>), dim3(a.grid), dim3(kWave * G), 0,
                               st, (const CT *)a.rowsA, (const CT *)a.rowsB, (int)a.nA, (int)a.nB,
                               CostArgs<CT>::make(cp), (Pair2<AT> *)a.bnd, a.flags, a.ticket, a.ticket + 1,
                               (int)a.nStrips, (const CT *)a.beta, (AT *)a.out, (AT *)a.dump, a.sub_shift, TileIO<AT>{});
            return hipGetLastError();
        } else {
            return hipErrorInvalidValue;
        }
    }
    hipLaunchKernelGGL((wavefront_kernel<CT, AT, DIMT, PM, K, G, false, false>), dim3(a.grid), dim3(kWave * G), 0, st,
                       (const CT *)a.rowsA, (const CT *)a.rowsB, (int)a.nA, (int)a.nB, CostArgs<CT>::make(cp),
                       (Pair2<AT> *)a.bnd, a.flags, a.ticket, a.ticket + 1, (int)a.nStrips, (const CT *)a.beta,
                       (AT *)a.out, nullptr, a.sub_shift, TileIO<AT>{});
    return hipGetLastError();
}

template <typename CT, typename AT, int DIMT, int PM, int K>
static hipError_t launch_k(const WavefrontArgs &a, const CostParams &cp, hipStream_t st)
{
    switch (a.group) {
    case 1: return launch_kg<CT, AT, DIMT, PM, K, 1>(a, cp, st);
    case 4: return launch_kg<CT, AT, DIMT, PM, K, 4>(a, cp, st);
    case 8: return launch_kg<CT, AT, DIMT, PM, K, 8>(a, cp, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename CT, int DIMT, int PM>
__global__ __launch_bounds__(64) void offset_kernel(const CT *__restrict__ rowsA, int nA,
                                                    const CT *__restrict__ rowsB, int nB, CostArgs<CT> ca,
                                                    CT *beta)
{
    const CT b = pair_offset<CT, DIMT, PM>(rowsA, nA, rowsB, nB, ca.nu, ca.p, ca.invp);
    beta[0] = b;  // every lane stores the same value
}

hipError_t launch_offset(Prec prec, const CostParams &cp, const void *rowsA, int64_t nA, const void *rowsB,
                         int64_t nB, void *beta, hipStream_t st)
{
    return by_prec(prec, cp.dimt, cp.pm, [&]<typename CT, typename AT, int DIMT, int PM>() -> hipError_t {
        hipLaunchKernelGGL((offset_kernel<CT, DIMT, PM>), dim3(1), dim3(kWave), 0, st, (const CT *)rowsA, (int)nA,
                           (const CT *)rowsB, (int)nB, CostArgs<CT>::make(cp), (CT *)beta);
        return hipGetLastError();
    });
}

hipError_t launch_wavefront(Prec prec, const CostParams &cp, int K, const WavefrontArgs &a, hipStream_t st)
{
    return by_prec(prec, cp.dimt, cp.pm, [&]<typename CT, typename AT, int DIMT, int PM>() -> hipError_t {
        switch (K) {
        case 1: return launch_k<CT, AT, DIMT, PM, 1>(a, cp, st);
        case 2: return launch_k<CT, AT, DIMT, PM, 2>(a, cp, st);
        case 4:
            if constexpr (kStripCompiled<DIMT, 4>) return launch_k<CT, AT, DIMT, PM, 4>(a, cp, st);
            return hipErrorInvalidValue;
        case 8:
            if constexpr (kStripCompiled<DIMT, 8>) return launch_k<CT, AT, DIMT, PM, 8>(a, cp, st);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
        }
    });
}

size_t wavefront_scratch_bytes(Prec prec, const CostParams &cp, int K, int G)
{
    size_t bytes = (size_t)-1;
    (void)by_prec(prec, cp.dimt, cp.pm, [&]<typename CT, typename AT, int DIMT, int PM>() -> hipError_t {
        auto pick = [&]<int KK>() -> size_t {
            switch (G) {
            case 1: return scratch_kg<CT, AT, DIMT, PM, KK, 1, false>();
            case 4: return scratch_kg<CT, AT, DIMT, PM, KK, 4, false>();
            case 8: return scratch_kg<CT, AT, DIMT, PM, KK, 8, false>();
            default: return (size_t)-1;
            }
        };
        switch (K) {
        case 1: bytes = pick.template operator()<1>(); break;
        case 2: bytes = pick.template operator()<2>(); break;
        case 4:
            if constexpr (kStripCompiled<DIMT, 4>) bytes = pick.template operator()<4>();
            break;
        case 8:
            if constexpr (kStripCompiled<DIMT, 8>) bytes = pick.template operator()<8>();
            break;
        default: break;
        }
        return hipSuccess;
    });
    return bytes;
}

int wavefront_max_workers(Prec prec, const CostParams &cp, int K, int G)
{
    int per_cu = 0;
    hipError_t e = by_prec(prec, cp.dimt, cp.pm, [&]<typename CT, typename AT, int DIMT, int PM>() -> hipError_t {
        switch (K) {
        case 1: per_cu = occupancy_k<CT, AT, DIMT, PM, 1, false>(G); break;
        case 2: per_cu = occupancy_k<CT, AT, DIMT, PM, 2, false>(G); break;
        case 4:
            if constexpr (kStripCompiled<DIMT, 4>) per_cu = occupancy_k<CT, AT, DIMT, PM, 4, false>(G);
            break;
        case 8:
            if constexpr (kStripCompiled<DIMT, 8>) per_cu = occupancy_k<CT, AT, DIMT, PM, 8, false>(G);
            break;
        default: break;
        }
        return hipSuccess;
    });
    if (e != hipSuccess || per_cu <= 0) return 0;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return per_cu * cus;
}

}  // namespace twed
