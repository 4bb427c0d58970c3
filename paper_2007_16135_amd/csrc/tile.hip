// tile.hip -- the sweep of one rectangular block of the DP matrix.
//
// The paper's section "Improved Time Warp Edit Distance" keeps only the band
// of live diagonals; a row or a column of (DP, X = DP + e) cells is likewise
// the whole state the rest of the program needs.  The tile sweep is the
// strip pipeline of wavefront.hip started from a given top row and left
// column instead of the pad row and column, and it can hand back its bottom
// row and right column, checkpoint rows and columns at fixed intervals, and
// the move taken into every cell.  Tiles in dependency order reproduce the
// pair sweep exactly: every cell is evaluated by the same lane code from the
// same operands.
//
// Tiles run with FP64 accumulators only (F64 and F32 costs with F64
// accumulators), where no cost offset is applied.
#include "wavefront_impl.h"

#include <type_traits>

namespace twed {

namespace {

template <typename CT, typename AT, int DIMT, int PM, int K, int G>
hipError_t launch_tile_kg(const WavefrontArgs &a, const TileIO<AT> &io, const CostParams &cp, hipStream_t st)
{
    hipLaunchKernelGGL((wavefront_kernel<CT, AT, DIMT, PM, K, G, false, true>), dim3(a.grid), dim3(kWave * G), 0, st,
                       (const CT *)a.rowsA, (const CT *)a.rowsB, (int)a.nA, (int)a.nB, CostArgs<CT>::make(cp),
                       (Pair2<AT> *)a.bnd, a.flags, a.ticket, a.ticket + 1, (int)a.nStrips, (const CT *)a.beta,
                       (AT *)a.out, nullptr, a.sub_shift, io);
    return hipGetLastError();
}

template <typename CT, typename AT, int DIMT, int PM, int K>
hipError_t launch_tile_k(const WavefrontArgs &a, const TileIO<AT> &io, const CostParams &cp, hipStream_t st)
{
    switch (a.group) {
    case 1: return launch_tile_kg<CT, AT, DIMT, PM, K, 1>(a, io, cp, st);
    case 4: return launch_tile_kg<CT, AT, DIMT, PM, K, 4>(a, io, cp, st);
    case 8: return launch_tile_kg<CT, AT, DIMT, PM, K, 8>(a, io, cp, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename AT>
TileIO<AT> typed(const TileArgs &t)
{
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
    return io;
}

// Cell 0 of each output row (column 0 of the block) and of each output
// column (row 0 of the block) is not on the strips: it is copied from the
// left column and the top row, or is the +inf pad cell.
__global__ void tile_edges_kernel(TileArgs t, int64_t nA, int64_t nB)
{
    typedef Pair2<double> C;
    const C inf{__builtin_inf(), __builtin_inf()};
    const C *top = (const C *)t.top, *left = (const C *)t.left;
    const int64_t nr = t.ckrow ? (nA - 1) / t.ck_rows : 0;   // checkpoint rows below nA
    const int64_t nc = t.ckcol ? (nB - 1) / t.ck_cols : 0;   // checkpoint columns left of nB
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nr + nc + 2;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (i == 0) {
            if (t.bottom) ((C *)t.bottom)[0] = left ? left[nA] : inf;
        } else if (i == 1) {
            if (t.right) ((C *)t.right)[0] = top ? top[nB] : inf;
        } else if (i - 2 < nr) {
            const int64_t r = (i - 1) * t.ck_rows;
            ((C *)t.ckrow)[(i - 2) * (nB + 1)] = left ? left[r] : inf;
        } else {
            const int64_t k = i - 2 - nr;
            const int64_t c = (k + 1) * t.ck_cols;
            ((C *)t.ckcol)[k * (nA + 1)] = top ? top[c] : inf;
        }
    }
}

}  // namespace

hipError_t launch_tile(Prec prec, const CostParams &cp, int K, const WavefrontArgs &a, const TileArgs &t,
                       hipStream_t st)
{
    if (prec != kF64 && prec != kF32Acc64) return hipErrorInvalidValue;
    if (t.dirs) return launch_tile_dirs(prec, cp, K, a, t, st);
    hipError_t e = by_prec(prec, cp.dimt, cp.pm, [&]<typename CT, typename AT, int DIMT, int PM>() -> hipError_t {
        if constexpr (!std::is_same_v<AT, double>) {
            return hipErrorInvalidValue;
        } else {
            const TileIO<AT> io = typed<AT>(t);
            switch (K) {
            case 1: return launch_tile_k<CT, AT, DIMT, PM, 1>(a, io, cp, st);
            case 2: return launch_tile_k<CT, AT, DIMT, PM, 2>(a, io, cp, st);
            case 4:
                if constexpr (kStripCompiled<DIMT, 4>) return launch_tile_k<CT, AT, DIMT, PM, 4>(a, io, cp, st);
                return hipErrorInvalidValue;
            case 8:
                if constexpr (kStripCompiled<DIMT, 8>) return launch_tile_k<CT, AT, DIMT, PM, 8>(a, io, cp, st);
                return hipErrorInvalidValue;
            default: return hipErrorInvalidValue;
            }
        }
    });
    if (e != hipSuccess) return e;
    return launch_tile_edges(a.nA, a.nB, t, st);
}

hipError_t launch_tile_edges(int64_t nA, int64_t nB, const TileArgs &t, hipStream_t st)
{
    if (!(t.bottom || t.right || t.ckrow || t.ckcol)) return hipSuccess;
    hipLaunchKernelGGL(tile_edges_kernel, dim3(64), dim3(256), 0, st, t, nA, nB);
    return hipGetLastError();
}

size_t tile_scratch_bytes(Prec prec, const CostParams &cp, int K, int G)
{
    size_t bytes = (size_t)-1;
    if (prec != kF64 && prec != kF32Acc64) return bytes;
    (void)by_prec(prec, cp.dimt, cp.pm, [&]<typename CT, typename AT, int DIMT, int PM>() -> hipError_t {
        if constexpr (std::is_same_v<AT, double>) {
            auto pick = [&]<int KK>() -> size_t {
                switch (G) {
                case 1: return scratch_kg<CT, AT, DIMT, PM, KK, 1, true>();
                case 4: return scratch_kg<CT, AT, DIMT, PM, KK, 4, true>();
                case 8: return scratch_kg<CT, AT, DIMT, PM, KK, 8, true>();
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
        }
        return hipSuccess;
    });
    return bytes;
}

int tile_max_workers(Prec prec, const CostParams &cp, int K, int G)
{
    int per_cu = 0;
    if (prec != kF64 && prec != kF32Acc64) return 0;
    (void)by_prec(prec, cp.dimt, cp.pm, [&]<typename CT, typename AT, int DIMT, int PM>() -> hipError_t {
        if constexpr (std::is_same_v<AT, double>) {
            switch (K) {
            case 1: per_cu = occupancy_k<CT, AT, DIMT, PM, 1, true>(G); break;
            case 2: per_cu = occupancy_k<CT, AT, DIMT, PM, 2, true>(G); break;
            case 4:
                if constexpr (kStripCompiled<DIMT, 4>) per_cu = occupancy_k<CT, AT, DIMT, PM, 4, true>(G);
                break;
            case 8:
                if constexpr (kStripCompiled<DIMT, 8>) per_cu = occupancy_k<CT, AT, DIMT, PM, 8, true>(G);
                break;
            default: break;
            }
        }
        return hipSuccess;
    });
    if (per_cu <= 0) return 0;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return per_cu * cus;
}

}  // namespace twed
