// Finite-difference constants of the Z4c kernels, as exact rationals.
//
// Order 2N centred operators on the points -N..N (Sec. 3: differencing of
// order 2(N_g - 1); Sec. 4.3: 6th order by default), written for the
// difference forms the kernels evaluate:
//   d/dx   f ~ (1/h)   sum_{k=1..N} D1[k] (f_k - f_-k)
//   d2/dx2 f ~ (1/h^2) sum_{k=1..N} D2[k] ((f_k - f_0) + (f_-k - f_0))
// The lopsided (upwind-biased) first derivative for a positive advection
// speed uses the points -(N-1)..N+1 (LOP, index k + N - 1); its mirror
// image serves negative speeds.  The kernels split it into its odd part
// (ODD[k], acting on f_k - f_-k) and even part (EVEN[k], acting on
// f_k + f_-k - 2 f_0), so that  v L_sign(v) f = v*odd + |v|*even.
// Kreiss-Oliger dissipation with r = N+1:
//   sigma (-1)^(r+1) 2^(-2r) (1/h) sum_axes Delta^r f
//   = (sigma/h) sum_axes sum_{k=1..r} KO[k] ((f_k - f_0) + (f_-k - f_0)).
#pragma once

namespace z4c {

template <int N> struct Stencil;

template <> struct Stencil<2> {
    static constexpr double D1[3] = {0.0, 2.0 / 3.0, -1.0 / 12.0};
    static constexpr double D2[3] = {-5.0 / 2.0, 4.0 / 3.0, -1.0 / 12.0};
    static constexpr double LOP[5] = {-1.0 / 4.0, -5.0 / 6.0, 3.0 / 2.0, -1.0 / 2.0, 1.0 / 12.0};
    static constexpr double KO[4] = {0.0, 15.0 / 64.0, -6.0 / 64.0, 1.0 / 64.0};
};

template <> struct Stencil<3> {
    static constexpr double D1[4] = {0.0, 3.0 / 4.0, -3.0 / 20.0, 1.0 / 60.0};
    static constexpr double D2[4] = {-49.0 / 18.0, 3.0 / 2.0, -3.0 / 20.0, 1.0 / 90.0};
    static constexpr double LOP[7] = {1.0 / 30.0, -2.0 / 5.0, -7.0 / 12.0, 4.0 / 3.0,
                                      -1.0 / 2.0, 2.0 / 15.0, -1.0 / 60.0};
    static constexpr double KO[5] = {0.0, 56.0 / 256.0, -28.0 / 256.0, 8.0 / 256.0, -1.0 / 256.0};
};

template <> struct Stencil<4> {
    static constexpr double D1[5] = {0.0, 4.0 / 5.0, -1.0 / 5.0, 4.0 / 105.0, -1.0 / 280.0};
    static constexpr double D2[5] = {-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0,
                                     -1.0 / 560.0};
    static constexpr double LOP[9] = {-1.0 / 168.0, 1.0 / 14.0, -1.0 / 2.0, -9.0 / 20.0, 5.0 / 4.0,
                                      -1.0 / 2.0, 1.0 / 6.0, -1.0 / 28.0, 1.0 / 280.0};
    static constexpr double KO[6] = {0.0, 210.0 / 1024.0, -120.0 / 1024.0, 45.0 / 1024.0,
                                     -10.0 / 1024.0, 1.0 / 1024.0};
};

// weight of the (+) lopsided operator at offset m (0 outside its support)
template <int N> __host__ __device__ constexpr double lop_w(int m)
{
    return (m >= -(N - 1) && m <= N + 1) ? Stencil<N>::LOP[m + N - 1] : 0.0;
}
// odd and even parts of the lopsided operator, k = 1..N+1
template <int N> __host__ __device__ constexpr double lop_odd(int k)
{
    return 0.5 * (lop_w<N>(k) - lop_w<N>(-k));
}
template <int N> __host__ __device__ constexpr double lop_even(int k)
{
    return 0.5 * (lop_w<N>(k) + lop_w<N>(-k));
}

}  // namespace z4c
