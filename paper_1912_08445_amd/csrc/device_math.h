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

// 2^{j/16}, j = 0..15, correctly rounded: the table of exp_tab16 (copied into LDS by the
// kernels that use it).
constexpr double kExp2Sixteenths[16] = {
    0x1.0000000000000p+0, 0x1.0b5586cf9890fp+0, 0x1.172b83c7d517bp+0, 0x1.2387a6e756238p+0,
    0x1.306fe0a31b715p+0, 0x1.3dea64c123422p+0, 0x1.4bfdad5362a27p+0, 0x1.5ab07dd485429p+0,
    0x1.6a09e667f3bcdp+0, 0x1.7a11473eb0187p+0, 0x1.8ace5422aa0dbp+0, 0x1.9c49182a3f090p+0,
    0x1.ae89f995ad3adp+0, 0x1.c199bdd85529cp+0, 0x1.d5818dcfba487p+0, 0x1.ea4afa2a490dap+0};

// e^y for y <= 700 in FP64, table-driven: y = (16 e + j) ln2/16 + r with |r| <= ln2/32
// (two-part ln2/16), e^y = 2^e 2^{j/16} e^r, e^r by its degree-7 Taylor polynomial
// (truncation < 2e-18 relative), tab = kExp2Sixteenths.  Below -745.2 the result is 0
// (y is first raised to -760, whose value is 0 after the scaling).  Within 2 ulp.  Fewer
// constants than exp_le700, which matters in register-bound kernels.
__device__ __forceinline__ double exp_tab16(double y, const double *tab)
{
    y = fmax(y, -760.0);
    const double n = rint(y * 0x1.71547652b82fep+4);       // 16 / ln2
    double r = fma(-n, 0x1.62e42ff000000p-5, y);           // ln2/16, leading 32 bits
    r = fma(-n, -0x1.718432a1b0e26p-39, r);                // the rest of ln2/16
    double p = 0x1.a01a01a01a01ap-13;                      // 1/7!
    p = fma(p, r, 0x1.6c16c16c16c17p-10);                  // 1/6!
    p = fma(p, r, 0x1.1111111111111p-7);                   // 1/5!
    p = fma(p, r, 0x1.5555555555555p-5);                   // 1/4!
    p = fma(p, r, 0x1.5555555555555p-3);                   // 1/3!
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    const int ni = (int)n;
    return ldexp(tab[ni & 15] * p, ni >> 4);
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
