// twed_dispatch.h -- maps a runtime (precision, compiled dimension, Lp mode)
// triple onto the matching kernel template instantiation.
#pragma once

#include "twed_device.h"
#include "twed_kernels.h"

namespace twed {

template <typename CT, typename AT, int DIMT, typename Fn>
hipError_t by_pm(int pm, Fn &&fn)
{
    if constexpr (DIMT == 1) {
        return fn.template operator()<CT, AT, DIMT, kL1>();
    } else {
        switch (pm) {
        case kL1: return fn.template operator()<CT, AT, DIMT, kL1>();
        case kL2: return fn.template operator()<CT, AT, DIMT, kL2>();
        default: return fn.template operator()<CT, AT, DIMT, kLp>();
        }
    }
}

template <typename CT, typename AT, typename Fn>
hipError_t by_dim(int dimt, int pm, Fn &&fn)
{
    switch (dimt) {
    case 1: return by_pm<CT, AT, 1>(pm, fn);
    case 2: return by_pm<CT, AT, 2>(pm, fn);
    case 3: return by_pm<CT, AT, 3>(pm, fn);
    case 4: return by_pm<CT, AT, 4>(pm, fn);
    case 8: return by_pm<CT, AT, 8>(pm, fn);
    case 16: return by_pm<CT, AT, 16>(pm, fn);
    case 32: return by_pm<CT, AT, 32>(pm, fn);
    default: return hipErrorInvalidValue;
    }
}

template <typename Fn>
hipError_t by_prec(Prec prec, int dimt, int pm, Fn &&fn)
{
    switch (prec) {
    case kF64: return by_dim<double, double>(dimt, pm, fn);
    case kF32: return by_dim<float, float>(dimt, pm, fn);
    case kF32Acc64: return by_dim<float, double>(dimt, pm, fn);
    default: return hipErrorInvalidValue;
    }
}

// Launch-shaped view of the cost parameters in the cost type.
template <typename CT>
struct CostArgs {
    CT nu, lambda, p, invp;
    static CostArgs make(const CostParams &cp)
    {
        return CostArgs{(CT)cp.nu, (CT)cp.lambda, (CT)cp.p, (CT)(1.0 / cp.p)};
    }
};

}  // namespace twed
