// General bound kernel: one lane per node, 32-bit arithmetic, any instance
// that passes fsp_create_instance (values below 2^31).
//
// For each machine pair (k,l) (Fig. 2), the lane walks the pair's
// Johnson-with-lags order (the JM row, the same for every node, so every
// record is a wave-uniform scalar load) and updates only for unscheduled jobs.
// The update of Fig. 2 (timeOnM1 += a; timeOnM2 = max(timeOnM2, timeOnM1 +
// lag) + b) is carried as the gap s = timeOnM2 - timeOnM1:
//     s <- max(s, lag + a) + (b - a),
// because timeOnM1 at the end of the scan is the release of k plus the time
// of all unscheduled jobs on k, known from the decode.  The select for
// scheduled jobs is one bitwise op on a mask taken from the register-resident
// bit set of unscheduled jobs.
#include "bound_common.h"

namespace fspbb {

template <int MV>
__global__ __launch_bounds__(256) void bound_lane32_kernel(DevTables T, const int32_t *__restrict__ prefixes,
                                                           const int32_t *__restrict__ depths, int64_t N,
                                                           int32_t *__restrict__ out_lb)
{
    __shared__ uint32_t bits[kMaskWords * 256];
    const int tid = threadIdx.x;
    const int64_t node = (int64_t)blockIdx.x * 256 + tid;
    const bool live = node < N;
    const int n = T.n;
    const int d = live ? depths[node] : 0;
    Decoded<MV> D;
    decode_node<MV>(T, prefixes + (live ? node : 0) * (int64_t)n, d, bits + tid, 256, D);

    constexpr int VW = MV < 16 ? 16 : MV;  // register vectors the compiler indexes with one move
    i32v<VW> R, TK, QV;
#pragma unroll
    for (int k = 0; k < VW; ++k) {
        R[k] = k < MV ? D.R[k] : 0;
        TK[k] = k < MV ? D.Tk[k] : 0;
        QV[k] = k < MV ? D.Qv[k] : 0;
    }
    const u32v<kMaskWords> act = D.act;

    int32_t lb = 0;
    for (int pr = 0; pr < T.P; ++pr) {
        const int k = as_const(T.pairs)[2 * pr], l = as_const(T.pairs)[2 * pr + 1];
        int32_t s = R[l] - R[k];
        cptr<int32_t> rec = as_const(reinterpret_cast<const int32_t *>(T.rec32 + (size_t)pr * n));
#pragma unroll 4
        for (int i = 0; i < n; ++i) {
            const int32_t word = rec[4 * i], bit = rec[4 * i + 1], E = rec[4 * i + 2], C = rec[4 * i + 3];
            const int32_t msk = __builtin_amdgcn_sbfe((int32_t)act[word], bit, 1);
            const int32_t t = max(s, E) + C;
            s = (msk & t) | (~msk & s);
        }
        lb = max(lb, TK[k] + s + QV[l]);
    }
    if (live) {
        out_lb[node] = D.ok ? lb : FSP_LB_INVALID;
        if (!D.ok) atomicAdd(T.bad, 1ull);
    }
}

hipError_t launch_bound_lane32(fsp_instance_s *I, const int32_t *prefixes, const int32_t *depths,
                               int64_t N, int32_t *out_lb, hipStream_t s)
{
    if (N <= 0) return hipSuccess;
    const dim3 grid((unsigned)((N + 255) / 256)), block(256);
    timing_mark(I, 0, s);
    timing_mark(I, 1, s);  // no separate decode kernel: the decode share counts as scan
    if (I->m <= 8)
        bound_lane32_kernel<8><<<grid, block, 0, s>>>(I->dt, prefixes, depths, N, out_lb);
    else if (I->m <= 16)
        bound_lane32_kernel<16><<<grid, block, 0, s>>>(I->dt, prefixes, depths, N, out_lb);
    else
        bound_lane32_kernel<32><<<grid, block, 0, s>>>(I->dt, prefixes, depths, N, out_lb);
    timing_mark(I, 2, s);
    return hipGetLastError();
}

}  // namespace fspbb
