// FP64 kernels of the polynomial orders 9..12 (the orders above the FP32
// maximum), in a translation unit of their own so that they compile in
// parallel with the others.  SkLaunch<double> routes these orders here.
#include "sk_launch_impl.h"

#define SK_HI_CASES(CALL) \
    case 9: return CALL(9); \
    case 10: return CALL(10); \
    case 11: return CALL(11); \
    case 12: return CALL(12); \
    default: return hipErrorInvalidValue;

hipError_t sk_hi_sweep(const SweepArgs<double>& a, int N, bool interp, bool ckpt, int64_t npairs,
                       int ring, bool gx, hipStream_t st) {
#define SK_C(n) sk_sweep_t<double, n>(a, interp, ckpt, npairs, ring, gx, st)
    switch (N) { SK_HI_CASES(SK_C) }
#undef SK_C
}

hipError_t sk_hi_sweep_pipe(const PipeArgs<double>& a, int N, bool interp, bool ckpt, hipStream_t st) {
    constexpr int T = SkTailMax<double>::value;
#define SK_C(n) (interp ? sk_pipe_n<double, n, T>(a, ckpt, st) : sk_pipe_n<double, n, 0>(a, ckpt, st))
    switch (N) { SK_HI_CASES(SK_C) }
#undef SK_C
}

hipError_t sk_hi_adjoint(const AdjArgs<double>& a, int N, bool interp, int64_t npairs, int ring,
                         bool gx, hipStream_t st) {
#define SK_C(n) sk_adj_t<double, n>(a, interp, npairs, ring, gx, st)
    switch (N) { SK_HI_CASES(SK_C) }
#undef SK_C
}

hipError_t sk_hi_adjoint_pipe(const AdjPipeArgs<double>& a, int N, bool interp, hipStream_t st) {
    constexpr int T = SkTailMax<double>::value;
#define SK_C(n) (interp ? sk_adj_pipe_n<double, n, T>(a, st) : sk_adj_pipe_n<double, n, 0>(a, st))
    switch (N) { SK_HI_CASES(SK_C) }
#undef SK_C
}

hipError_t sk_hi_plain_poly(const PlainArgs<double>& a, int N, bool interp, hipStream_t st) {
#define SK_C(n) sk_plain_n<double, n>(a, interp, st)
    switch (N) { SK_HI_CASES(SK_C) }
#undef SK_C
}

// this unit's status word (its kernels raise their SK_STATUS_* bits here)
hipError_t sk_hi_status_word(unsigned** p) {
    return hipGetSymbolAddress(reinterpret_cast<void**>(p), HIP_SYMBOL(sk_status_word));
}
