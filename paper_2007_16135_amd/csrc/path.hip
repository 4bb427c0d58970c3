// path.hip -- reading an optimal alignment path back from recorded moves.
//
// The paper's section "Time Warp Edit Distance" notes that the alignment
// path follows by backtracking over the choices of the forward problem.  The
// tile sweep records the move into every cell of a block (one byte, in sweep
// order) and the walk below follows them from a cell of the block back to the
// block's top row or left column.  The path is written from its end, (nA, nB), so
// the cells come out in reverse; a last pass puts them in order.
#include "twed_device.h"
#include "twed_kernels.h"

namespace twed {

namespace {

// One wave.  The walk is a chain of dependent reads, so the moves of the 64 x
// 64 cells up and to the left of the current cell are first gathered into
// LDS (lane l reads one column, 64 rows: every row of a column sits 64*K
// bytes after the previous one in sweep order), and the walk then follows
// them there until it leaves that window.  Every lane runs the same walk
// (uniform control flow) and stores the same cells.  st = {r, c, n, status}
// in global coordinates; status 0 running, 1 reached (0, 0), -1 failed.
//
// With free_edges (edit and indel distances, whose row 0 and column 0 are
// finite) a walk that reaches row 0 or column 0 follows it to (0, 0); for
// TWED and DTW those cells are +inf and reaching one is an error.
__global__ __launch_bounds__(kWave) void walk_kernel(const uint8_t *__restrict__ dirs, int64_t r0, int64_t c0,
                                                     int64_t nAt, int64_t nBt, int K, int64_t T, int64_t *st,
                                                     int64_t *rev, int64_t cap, int free_edges)
{
    __shared__ uint8_t win[kWave * kWave];
    const int lane = threadIdx.x;
    if (st[3] != 0) return;
    int64_t r = st[0], c = st[1], n = st[2];
    int64_t status = 0;
    const int64_t W = (int64_t)kWave * K;
    for (;;) {
        if (r == 0 || c == 0) {
            if (!(r == 0 && c == 0) && !free_edges) {
                status = -1;
                break;
            }
            while (n < cap) {
                rev[2 * n] = r;
                rev[2 * n + 1] = c;
                ++n;
                if (r == 0 && c == 0) break;
                if (r > 0) --r;
                else --c;
            }
            status = (r == 0 && c == 0) ? 1 : -1;
            break;
        }
        const int64_t rr = r - r0, cc = c - c0;
        if (rr <= 0 || cc <= 0) break;  // the cell belongs to the block above or to the left
        // window of local rows wr..rr and columns wc..cc
        const int64_t wr = rr - (kWave - 1), wc = cc - (kWave - 1);
        __syncthreads();  // the previous window has been read
        {
            int64_t col = wc + lane;
            col = col < 1 ? 1 : (col > nBt ? nBt : col);
            const int64_t s = (col - 1) / W, within = (col - 1) - s * W;
            const int64_t ln = within / K, j = within - ln * K;
            for (int k = 0; k < kWave; ++k) {
                int64_t row = wr + k;
                row = row < 1 ? 1 : (row > nAt ? nAt : row);
                win[k * kWave + lane] = dirs[((s * T + row + ln) * kWave + ln) * K + j];
            }
        }
        __syncthreads();
        for (;;) {
            const int64_t lr = r - r0, lc = c - c0;
            if (r == 0 || c == 0 || lr <= 0 || lc <= 0 || lr < wr || lc < wc) break;
            if (n >= cap) {
                status = -1;
                break;
            }
            rev[2 * n] = r;
            rev[2 * n + 1] = c;
            ++n;
            const uint8_t mv = win[(lr - wr) * kWave + (lc - wc)];
            if (mv == 0) {
                --r;
                --c;
            } else if (mv == 1) {
                --r;
            } else if (mv == 2) {
                --c;
            } else {
                status = -1;
                break;
            }
        }
        if (status != 0) break;
    }
    st[0] = r;  // every lane stores the same values
    st[1] = c;
    st[2] = n;
    st[3] = status;
}

// path[k] = rev[n - 1 - k] for the n cells, and *len = n (0 on failure).
__global__ void order_kernel(const int64_t *st, int64_t *path, int64_t *len)
{
    const int64_t n = st[3] == 1 ? st[2] : 0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n / 2; k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t a = k, b = n - 1 - k;
        const int64_t ai = path[2 * a], aj = path[2 * a + 1];
        path[2 * a] = path[2 * b];
        path[2 * a + 1] = path[2 * b + 1];
        path[2 * b] = ai;
        path[2 * b + 1] = aj;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *len = n;
}

__global__ void walk_init_kernel(int64_t *st, int64_t nA, int64_t nB)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st[0] = nA;
        st[1] = nB;
        st[2] = 0;
        st[3] = 0;
    }
}

}  // namespace

hipError_t launch_walk_init(int64_t *st, int64_t nA, int64_t nB, hipStream_t s)
{
    hipLaunchKernelGGL(walk_init_kernel, dim3(1), dim3(1), 0, s, st, nA, nB);
    return hipGetLastError();
}

hipError_t launch_walk(const uint8_t *dirs, int64_t r0, int64_t c0, int64_t nAt, int64_t nBt, int K, int64_t T,
                       int64_t *st, int64_t *rev, int64_t cap, bool free_edges, hipStream_t s)
{
    hipLaunchKernelGGL(walk_kernel, dim3(1), dim3(kWave), 0, s, dirs, r0, c0, nAt, nBt, K, T, st, rev, cap,
                       free_edges ? 1 : 0);
    return hipGetLastError();
}

namespace {
// cells[i] = (i, i): row 0 or column 0 of the edit and indel distances.
__global__ void index_cells_kernel(double *cells, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += (int64_t)gridDim.x * blockDim.x) {
        cells[2 * i] = (double)i;
        cells[2 * i + 1] = (double)i;
    }
}

// LCS length from the indel distance: (nA + nB - I) / 2.
__global__ void lcs_finish_kernel(double *out, int64_t nA, int64_t nB)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) out[0] = ((double)(nA + nB) - out[0]) * 0.5;
}
}  // namespace

hipError_t launch_index_cells(void *cells, int64_t n, hipStream_t s)
{
    int64_t g = (n + 256) / 256;
    if (g > 1024) g = 1024;
    hipLaunchKernelGGL(index_cells_kernel, dim3((int)g), dim3(256), 0, s, (double *)cells, n);
    return hipGetLastError();
}

hipError_t launch_lcs_finish(double *out, int64_t nA, int64_t nB, hipStream_t s)
{
    hipLaunchKernelGGL(lcs_finish_kernel, dim3(1), dim3(1), 0, s, out, nA, nB);
    return hipGetLastError();
}

hipError_t launch_order(const int64_t *st, int64_t *path, int64_t *len, int64_t cap, hipStream_t s)
{
    int64_t g = (cap / 2 + 255) / 256;
    if (g < 1) g = 1;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(order_kernel, dim3((int)g), dim3(256), 0, s, st, path, len);
    return hipGetLastError();
}

}  // namespace twed

namespace twed {

namespace {
__global__ void zero32_kernel(uint32_t *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}
}  // namespace

hipError_t launch_zero32(uint32_t *p, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int64_t g = (n + 255) / 256;
    if (g > 1024) g = 1024;
    hipLaunchKernelGGL(zero32_kernel, dim3((int)g), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace twed
