// FP64 device arithmetic shared by the kernels (exponentials and a reciprocal without
// the library's special-case handling, for arguments these kernels produce).
#pragma once
#include <hip/hip_runtime.h>

namespace nlte {

// e^y for y <= 700 in FP64: y = n ln2 + r with |r| <= ln2/2 (two-part ln2), e^r by its
// degree-11 Taylor polynomial (truncation < 7e-15 relative), scaled by 2^n.  Results
// below the FP64 range come out as 0 through ldexp; no other special cases arise for
// the arguments used here (finite, at most 700).
__device__ __forceinline__ double exp_le700(double y)
{
    const double n = rint(y * 1.44269504088896338700);
    double r = fma(-n, 6.93147180369123816490e-01, y);
    r = fma(-n, 1.90821492927058770002e-10, r);
    double p = 2.50521083854417187751e-08;           // 1/11!
    p = fma(p, r, 2.75573192239858906526e-07);       // 1/10!
    p = fma(p, r, 2.75573192239858906526e-06);       // 1/9!
    p = fma(p, r, 2.48015873015873015873e-05);       // 1/8!
    p = fma(p, r, 1.98412698412698412698e-04);       // 1/7!
    p = fma(p, r, 1.38888888888888888889e-03);       // 1/6!
    p = fma(p, r, 8.33333333333333333333e-03);       // 1/5!
    p = fma(p, r, 4.16666666666666666667e-02);       // 1/4!
    p = fma(p, r, 1.66666666666666666667e-01);       // 1/3!
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    const int ni = (int)fmax(n, -2200.0);
    return ldexp(p, ni);
}

// e^{-u} for 0 <= u <= 0.5 by its degree-13 Taylor polynomial (truncation < 1e-15).
__device__ __forceinline__ double exp_neg_small(double u)
{
    double p = -1.60590438368216145994e-10;          // -1/13!
    p = fma(p, u, 2.08767569878680989792e-09);       // 1/12!
    p = fma(p, u, -2.50521083854417187751e-08);
    p = fma(p, u, 2.75573192239858906526e-07);
    p = fma(p, u, -2.75573192239858906526e-06);
    p = fma(p, u, 2.48015873015873015873e-05);
    p = fma(p, u, -1.98412698412698412698e-04);
    p = fma(p, u, 1.38888888888888888889e-03);
    p = fma(p, u, -8.33333333333333333333e-03);
    p = fma(p, u, 4.16666666666666666667e-02);
    p = fma(p, u, -1.66666666666666666667e-01);
    p = fma(p, u, 0.5);
    p = fma(p, u, -1.0);
    return fma(p, u, 1.0);
}

// 1/x for a normal positive x: the hardware estimate refined by two Newton steps
// (relative error near 1 ulp; not correctly rounded).
__device__ __forceinline__ double rcp_refined(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}

}  // namespace nlte
