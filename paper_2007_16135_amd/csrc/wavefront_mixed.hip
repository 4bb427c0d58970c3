// wavefront_mixed.hip -- the single-pair strip sweep with strips of two widths.
//
// A strip of 64*K columns starts one pipeline lag (64 + the in-group handoff
// interval, in its own steps) after the strip on its left and then runs
// nA + 63 steps of K cells per lane.  With every strip resident, the sweep
// ends when the last strip does, and uniform strips end in the order they
// start: the workgroups of the first strips idle through the tail of the
// sweep.  Narrowing the strips on the right (K on the left, K - 1 on the
// right) shortens the last strips' runs and puts the workgroup slots that
// uniform strips would leave empty to work.  Which strip switches width is
// chosen on the host from the pipeline's timing (choose_mixed_split).
//
// The layouts compiled (kMixedLayouts): strips of 8 and 7 columns in groups
// of eight waves, two waves per SIMD, for L1 and L2 distances and samples of
// up to eight components.  (Strips of 6 and 5 columns in groups of twelve,
// three waves per SIMD, ran the 8-D pair of 1e6 samples 14% slower: the
// SIMD's issue rate is already spent with two waves of this instruction mix,
// so the third wave only slows the other two, and the pipeline fill grows.)
#include "wavefront_impl.h"

namespace twed {

template <int DIMT, int PM>
constexpr bool kMixedCompiled = DIMT <= 8 && PM != kLp;

// fn.template operator()<CT, AT, DIMT, PM, M>() for the compiled combination,
// or hipErrorInvalidValue.
template <typename Fn>
hipError_t by_layout(Prec prec, const CostParams &cp, int layout, Fn &&fn)
{
    return by_prec(prec, cp.dimt, cp.pm, [&]<typename CT, typename AT, int DIMT, int PM>() -> hipError_t {
        if constexpr (kMixedCompiled<DIMT, PM>) {
            switch (layout) {
            case 0: return fn.template operator()<CT, AT, DIMT, PM, 0>();
            default: return hipErrorInvalidValue;
            }
        } else {
            return hipErrorInvalidValue;
        }
    });
}

template <typename CT, typename AT, int DIMT, int PM, int M>
constexpr auto mixed_kernel()
{
    constexpr MixedLayout L = kMixedLayouts[M];
    return wavefront_mixed_kernel<CT, AT, DIMT, PM, L.wide, L.narrow, L.group>;
}

bool wavefront_mixed_compiled(Prec prec, const CostParams &cp, int layout)
{
    return by_layout(prec, cp, layout, [&]<typename CT, typename AT, int DIMT, int PM, int M>() -> hipError_t {
               return hipSuccess;
           }) == hipSuccess;
}

hipError_t launch_wavefront_mixed(Prec prec, const CostParams &cp, int layout, const WavefrontArgs &a,
                                  hipStream_t st)
{
    if (layout < 0 || layout >= kNumMixedLayouts || a.group != kMixedLayouts[layout].group || a.s1 <= 0 ||
        a.dump != nullptr)
        return hipErrorInvalidValue;
    return by_layout(prec, cp, layout, [&]<typename CT, typename AT, int DIMT, int PM, int M>() -> hipError_t {
        hipLaunchKernelGGL((mixed_kernel<CT, AT, DIMT, PM, M>()), dim3(a.grid), dim3(kWave * kMixedLayouts[M].group),
                           0, st, (const CT *)a.rowsA, (const CT *)a.rowsB, (int)a.nA, (int)a.nB,
                           CostArgs<CT>::make(cp), (Pair2<AT> *)a.bnd, a.flags, a.ticket, a.ticket + 1,
                           (int)a.nStrips, a.s1, (const CT *)a.beta, (AT *)a.out, a.sub_shift);
        return hipGetLastError();
    });
}

int wavefront_mixed_max_workers(Prec prec, const CostParams &cp, int layout)
{
    int per_cu = 0;
    hipError_t e = by_layout(prec, cp, layout, [&]<typename CT, typename AT, int DIMT, int PM, int M>() -> hipError_t {
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, mixed_kernel<CT, AT, DIMT, PM, M>(),
                                                            kWave * kMixedLayouts[M].group, 0);
    });
    if (e != hipSuccess || per_cu <= 0) return 0;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return per_cu * cus;
}

size_t wavefront_mixed_scratch_bytes(Prec prec, const CostParams &cp, int layout)
{
    size_t bytes = (size_t)-1;
    (void)by_layout(prec, cp, layout, [&]<typename CT, typename AT, int DIMT, int PM, int M>() -> hipError_t {
        hipFuncAttributes attr{};
        if (hipFuncGetAttributes(&attr, reinterpret_cast<const void *>(mixed_kernel<CT, AT, DIMT, PM, M>())) ==
            hipSuccess)
            bytes = attr.localSizeBytes;
        return hipSuccess;
    });
    return bytes;
}

}  // namespace twed
