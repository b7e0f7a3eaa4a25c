// HIP kernel templates of the SCF hot path for gfx950 (MI355X), and the
// engine that launches them for one (dtype, nmax bound, lmax).  Included by
// the translation units that instantiate the engines.
//
// Coefficient pass (Sec. 2, Eq. sumanlm): a_t = -sum_k m_k psi*_t(x_k) is a
// sum over particles of an outer product, per degree l, of the radial vector
// m_k G_l p_n^(l)(xi_k) (n = 0..nmax) and the angular vector
// Qt_l^m(c_k) {Re, Im}(u_k^m) (j = 0..2l).  One wave per block:
//   1. basis phase: the wave evaluates both vectors for a stage of P particles
//      (LPP lanes per particle, split by l and m residues) into a private LDS
//      record per particle;
//   2. accumulation phase: every lane owns a register tile of NR rows (n) x JT
//      columns (j) of one l-block and sweeps the staged particles, so each LDS
//      operand feeds NR*JT/(NR+JT) fused multiply-adds.  G lane groups take
//      disjoint subsets of the stage when the tiles need fewer than 64 lanes.
//   Each block writes one partial per coefficient; a second pass sums the
//   partials over blocks in double precision in a fixed order.
// Field pass (Eq. total_potential and its gradient): one particle per lane; the
// force weights W_t (coefficients times normalisations) are wave-uniform and
// are read with scalar loads, the radial sums sigma_lj = sum_n W_nlj p_n and
// their xi-derivatives take 2 FMAs per particle-term, and the angular sums
// follow from the same monic Legendre recurrence, its derivative and u^m.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdio>
#include <type_traits>

#include "scf_device.h"
#include "scf_internal.h"

namespace scf {

constexpr int ceil_div_c(int a, int b) { return (a + b - 1) / b; }
constexpr int ntiles_c(int lmax, int jt) {
  int s = 0;
  for (int l = 0; l <= lmax; ++l) s += ceil_div_c(2 * l + 1, jt);
  return s;
}

// Tile shape of the accumulation phase, chosen at compile time.  Each lane
// owns NR rows (n = 0..NMAXC) x JT columns (j) of one degree l and rebuilds the
// radial column p_n^(l)(xi) itself from two staged numbers (xi and m G_l), so
// the cost per staged particle is NR*JT FMAs plus 2(NR-2) recurrence ops; the
// model picks JT (and the number of lane groups G sharing a stage) under a
// register budget for the accumulators.
template <typename R, int NMAXC, int LMAX, int LPP_>
struct CoefShape {
  static constexpr int LPP = LPP_;
  static constexpr int P = 64 / LPP;
  static constexpr int NR = NMAXC + 1;
  // accumulators per lane: 96 for float and double (the double kernels run
  // at one wave per SIMD either way, and the wider tiles fill more lanes:
  // 192 against 240 us at nmax 16, lmax 10), 64 for the dual numbers of the
  // adjoint's gamma pass
  static constexpr int ACC_MAX = (sizeof(R) == 4 || std::is_same<R, double>::value) ? 96 : 64;
  struct Pick {
    int jt, g, kt;
  };
  static constexpr Pick pick() {
    Pick best{1, 1, ceil_div_c(ntiles_c(LMAX, 1), 64)};
    double bcost = 1e30;
    for (int jt = 1; jt <= 8; ++jt) {
      int nt = ntiles_c(LMAX, jt);
      int kt = ceil_div_c(nt, 64);
      if (kt * NR * jt > ACC_MAX) continue;
      int g = 1;
      if (kt == 1) {
        g = 64 / nt;
        if (g > P) g = P;
        if (g > 4) g = 4;
        if (g < 1) g = 1;
      }
      int ppl = ceil_div_c(P, g);
      double valu = double(kt) * ppl * (NR * jt + 2 * (NR > 2 ? NR - 2 : 0) + 2);
      double lds = double(kt) * ppl * (jt + 2) * (sizeof(R) / 4);
      double cost = valu + 0.75 * lds;
      if (cost < bcost) {
        bcost = cost;
        best = Pick{jt, g, kt};
      }
    }
    return best;
  }
  static constexpr Pick pk = pick();
  static constexpr int JT = pk.jt, G = pk.g, KT = pk.kt;
  static constexpr int NT = ntiles_c(LMAX, JT);
  static constexpr int GS = 64 / G;  // lanes per group: groups start on lane multiples of GS
  static constexpr int L1 = LMAX + 1;
  // per-particle record: [xi, m G_0 .. m G_LMAX, angular columns tile-padded]
  static constexpr int GOFF = 1;
  static constexpr int AOFF = 1 + L1;
  static constexpr int AL = JT * NT;
  static constexpr int DUMP = AOFF + AL;          // scratch slot for masked stores
  static constexpr int PS = (AOFF + AL + 1) | 1;  // odd stride
  static constexpr int KR = (LMAX + LPP) / LPP;   // orders per lane in the basis phase
  static constexpr int aoff(int l) { return AOFF + JT * (ntiles_c(l - 1, JT)); }
};

// One particle of a coefficient pass: position and weight (mass), or in the
// gamma pass of the adjoint the dual position x + eps escale e with weight 1.
template <typename R>
__device__ __forceinline__ void load_particle(const CoefArgs<R>& a, int64_t i, R& x, R& y, R& z,
                                              R& m) {
  if constexpr (RealTraits<R>::dual) {
    x = R(a.x[i], a.escale * a.ex[i]);
    y = R(a.y[i], a.escale * a.ey[i]);
    z = R(a.z[i], a.escale * a.ez[i]);
    m = R(1);
  } else {
    x = a.x[i];
    y = a.y[i];
    z = a.z[i];
    m = a.m[i];
  }
}

// Wave-local ordering of LDS traffic: every wave works in its own region.
template <int WPB>
__device__ __forceinline__ void stage_sync() {
  if constexpr (WPB == 1) {
    __syncthreads();
  } else {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

template <typename R, int NMAXC, int LMAX, int LPP, int WPB>
__global__ void __launch_bounds__(64 * WPB) coef_kernel(CoefArgs<R> a) {
  using S = CoefShape<R, NMAXC, LMAX, LPP>;
  using Sc = scalar_t<R>;
  using A = acc_t<R>;
  constexpr int P = S::P, NR = S::NR, JT = S::JT, G = S::G, KT = S::KT, KR = S::KR;
  constexpr int NT = S::NT, L1 = S::L1, PS = S::PS, DUMP = S::DUMP;
  constexpr int REG = P * PS;  // one wave's stage buffer
  // lane groups are combined through the stage buffer when it is large enough,
  // otherwise every group writes its own partial row
  constexpr bool LDS_COMBINE = G == 1 || NT * NR * JT <= P * PS;
  constexpr int ROWS = LDS_COMBINE ? 1 : G;
  static_assert(KT > 1 || NT <= S::GS, "a group's tiles must fit its lanes");
  __shared__ R lds_all[WPB * REG];

  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  R* rec = lds_all + wave * REG;
  for (int i = lane; i < REG; i += 64) rec[i] = R(0);  // padding columns stay zero

  // ---- tile ownership and the owned degrees' recurrence constants ----------
  int grp = 0;
  int tl[KT], tj[KT], tt[KT];
  bool tv[KT];
  Sc bl[KT][NR];
#pragma unroll
  for (int k = 0; k < KT; ++k) {
    int tau;
    if (KT == 1) {
      grp = lane / S::GS;
      tau = lane % S::GS;
      tv[k] = grp < G && tau < NT;
    } else {
      tau = lane + 64 * k;
      tv[k] = tau < NT;
    }
    int l = 0;
    int rem = tau;
    for (int ll = 0; ll <= LMAX; ++ll) {
      int nt = (2 * ll + 1 + JT - 1) / JT;
      if (rem < nt) {
        l = ll;
        break;
      }
      rem -= nt;
      l = ll;
    }
    tl[k] = tv[k] ? l : 0;
    tj[k] = tv[k] ? rem * JT : 0;
    tt[k] = tv[k] ? tau : 0;
#pragma unroll
    for (int n = 0; n < NR; ++n) bl[k][n] = a.beta_rad[tl[k] * NR + n];
  }

  A acc[KT][NR][JT];
#pragma unroll
  for (int k = 0; k < KT; ++k)
#pragma unroll
    for (int i = 0; i < NR; ++i)
#pragma unroll
      for (int j = 0; j < JT; ++j) acc[k][i][j] = A(0);

  // particle range of this wave-unit
  const int unit = blockIdx.x * WPB + wave;
  if constexpr (WPB > 1) {
    if (unit >= a.nunits) return;  // surplus wave of the last block (no block barriers follow)
  } else {
    if (unit >= a.nunits) return;
  }
  int64_t begin, end;
  int slot;
  if (a.seg_begin) {
    begin = a.seg_begin[unit];
    end = a.seg_end[unit];
    slot = a.seg_slot[unit];
  } else {
    begin = a.begin + (a.stages * unit / a.nunits) * P;
    end = a.begin + (a.stages * (unit + 1) / a.nunits) * P;
    if (end > a.n) end = a.n;
    slot = unit;
  }
  const int q = lane / LPP, h = lane % LPP;
  R* rp = rec + q * PS;
  stage_sync<WPB>();

  // prefetched particle of the first stage
  R nx = R(0), ny = R(0), nz = R(0), nm = R(0);
  {
    const int64_t gi = begin + q;
    if (q < P && gi < end) load_particle(a, gi, nx, ny, nz, nm);
  }
  for (int64_t base = begin; base < end; base += P) {
    // ---- basis phase: xi, m G_l and the angular columns ---------------------
    {
      const R x = nx, y = ny, z = nz, mk = nm;
      Geom<R> g = make_geom<R>(x, y, z, a.binv, a.alpha, a.inv_alpha, a.amode);
      if (h == 0) {
        rp[0] = g.xi;
        R Gl = mk * g.g0;
#pragma unroll
        for (int l = 0; l <= LMAX; ++l) {
          rp[S::GOFF + l] = Gl;
          Gl *= g.w;
        }
      }
      R er = R(1), ei = R(0);
      for (int t = 0; t < h; ++t) {
        R nr = er * g.ux - ei * g.uy;
        ei = er * g.uy + ei * g.ux;
        er = nr;
      }
      R sr = g.ux, si = g.uy;  // u^LPP
#pragma unroll
      for (int t = 1; t < LPP; ++t) {
        R nr = sr * g.ux - si * g.uy;
        si = sr * g.uy + si * g.ux;
        sr = nr;
      }
#pragma unroll
      for (int kk = 0; kk < KR; ++kk) {
        const int mm = h + kk * LPP;
        const bool mv = mm <= LMAX;
        const int mc = mv ? mm : LMAX;
        const int offc = mm > 0 ? 2 * mm - 1 : 0;
        const int offs = 2 * mm;
        const Sc m2 = Sc(mc) * Sc(mc);
        R Q0 = R(0), Q1 = R(0);
#pragma unroll
        for (int l = kk * LPP; l <= LMAX; ++l) {
          // gamma_lm = ((l-1)^2 - m^2) / ((2l-1)(2l-3)), used for l >= m+2
          const Sc cl = l >= 2 ? Sc(1) / Sc((2 * l - 1) * (2 * l - 3)) : Sc(0);
          const Sc gam = fma(-m2, cl, Sc((l - 1) * (l - 1)) * cl);
          const R qg = g.c * Q1 - gam * Q0;
          const R Q = (l == mm) ? R(1) : qg;
          Q0 = Q1;
          Q1 = Q;
          const bool ok = mv && l >= mm;
          const int ic = ok ? S::aoff(l) + offc : DUMP;
          const int is = (ok && mm > 0) ? S::aoff(l) + offs : DUMP;
          rp[is] = Q * ei;
          rp[ic] = Q * er;
        }
        R nr = er * sr - ei * si;
        ei = er * si + ei * sr;
        er = nr;
      }
    }
    stage_sync<WPB>();
    // prefetch the next stage's particle while accumulating
    {
      const int64_t gi = base + P + q;
      if (gi < end) {
        load_particle(a, gi, nx, ny, nz, nm);
      } else {
        nx = ny = nz = nm = R(0);
      }
    }
    // ---- accumulation phase ------------------------------------------------
#pragma unroll
    for (int k = 0; k < KT; ++k) {
      if (tv[k]) {
        const R* gb = rec + S::GOFF + tl[k];
        const R* ab = rec + S::AOFF + JT * tt[k];
        constexpr int PPL = (P + G - 1) / G;
#pragma unroll 2
        for (int ii = 0; ii < PPL; ++ii) {
          const int p = grp + G * ii;
          if (G * PPL == P || p < P) {
            const R xi = rec[p * PS];
            R p0 = gb[p * PS];
            R av[JT];
#pragma unroll
            for (int j = 0; j < JT; ++j) av[j] = ab[p * PS + j];
#pragma unroll
            for (int j = 0; j < JT; ++j) acc[k][0][j] = fma(p0, av[j], acc[k][0][j]);
            if constexpr (NR > 1) {
              R p1 = xi * p0;
#pragma unroll
              for (int j = 0; j < JT; ++j) acc[k][1][j] = fma(p1, av[j], acc[k][1][j]);
#pragma unroll
              for (int i = 2; i < NR; ++i) {
                const R p2 = fma(xi, p1, -bl[k][i] * p0);
#pragma unroll
                for (int j = 0; j < JT; ++j) acc[k][i][j] = fma(p2, av[j], acc[k][i][j]);
                p0 = p1;
                p1 = p2;
              }
            }
          }
        }
      }
    }
    stage_sync<WPB>();
  }

  // ---- combine lane groups (in rounds) and write this unit's partials -------
  if constexpr (G > 1 && LDS_COMBINE) {
    static_assert(sizeof(A) <= sizeof(R), "accumulators are combined in the stage buffer");
    A* recA = reinterpret_cast<A*>(rec);
    for (int gg = 1; gg < G; ++gg) {
      if (grp == gg && tv[0]) {
        A* dst = recA + tt[0] * NR * JT;
#pragma unroll
        for (int i = 0; i < NR; ++i)
#pragma unroll
          for (int j = 0; j < JT; ++j) dst[i * JT + j] = acc[0][i][j];
      }
      stage_sync<WPB>();
      if (grp == 0 && tv[0]) {
        const A* src = recA + tt[0] * NR * JT;
#pragma unroll
        for (int i = 0; i < NR; ++i)
#pragma unroll
          for (int j = 0; j < JT; ++j) acc[0][i][j] += src[i * JT + j];
      }
      stage_sync<WPB>();
    }
  }
  A* out = a.partials + ((int64_t)slot * ROWS + (LDS_COMBINE ? 0 : grp)) * a.T;
  constexpr int AL2 = L1 * L1;
#pragma unroll
  for (int k = 0; k < KT; ++k) {
    if (tv[k] && (grp == 0 || !LDS_COMBINE)) {
      const int l = tl[k];
#pragma unroll
      for (int i = 0; i < NR; ++i) {
        if (i <= a.nmax) {
#pragma unroll
          for (int j = 0; j < JT; ++j) {
            const int jj = tj[k] + j;
            if (jj <= 2 * l) out[i * AL2 + l * l + jj] = acc[k][i][j];
          }
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// field kernel: acceleration (and potential) at every particle; in step mode
// also the fused kick and drift
// ---------------------------------------------------------------------------
__device__ __forceinline__ double uniform_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
  const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ int64_t uniform_i64(int64_t v) {
  const int lo = __builtin_amdgcn_readfirstlane((int)(v & 0xffffffffll));
  const int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
  return ((int64_t)hi << 32) | (unsigned int)lo;
}

// psi_SCF and a = -grad psi_SCF at one point (zero force at the origin).
// R is float, double or Dual<T>; the tables (W, recurrence constants) are of
// the scalar type.  The degree loop is a real (wave-uniform) loop so that only
// one degree's radial vector is live.
// The sums of one point over the degrees [lo, hi] (RANGED) or all degrees:
// psi, its radial derivative psir, and the angular gradient (gx, gy, gz) of
// the form Gamma below.  The Legendre factors of degrees below lo are still
// swept (their recurrence feeds the next degrees).
template <typename R, int NMAXC, int LMAX, bool RANGED>
__device__ __forceinline__ void field_sums(const Geom<R>& g, const scalar_t<R>* __restrict__ W,
                                           const scalar_t<R>* __restrict__ bR,
                                           const scalar_t<R>* __restrict__ bA, const int lo,
                                           const int hi, R& psi, R& psir, R& gx, R& gy, R& gz) {
  using Sc = scalar_t<R>;
  constexpr int L1 = LMAX + 1, NW = NMAXC + 1;

  R Er[L1], Ei[L1];
  Er[0] = R(1);
  Ei[0] = R(0);
#pragma unroll
  for (int m = 1; m <= LMAX; ++m) {
    Er[m] = Er[m - 1] * g.ux - Ei[m - 1] * g.uy;
    Ei[m] = Er[m - 1] * g.uy + Ei[m - 1] * g.ux;
  }
  psi = R(0);
  psir = R(0);
  gx = R(0);
  gy = R(0);
  gz = R(0);
  R Gprev = R(0), Gl = g.g0;
  // Degrees in pairs: the Legendre factors of degree l overwrite those of
  // degree l-2 (two arrays in ping-pong fashion), and the orders are a static
  // sweep m = LMAX..0 that skips m > l, so every register array is statically
  // indexed.  One recurrence covers every order m <= l: each array starts as 1
  // at the indices of its own degree parity and 0 elsewhere, and the table
  // holds b_{m,m} = -1, so entries that no degree has written yet give
  // Qt_m^m = c 0 + 1 = 1 and Qt_{m+1}^m = c 1 - b 0 = c exactly.
  R QA[L1], QB[L1];
#pragma unroll
  for (int m = 0; m <= LMAX; ++m) {
    QA[m] = R((m & 1) == 0 ? 1 : 0);
    QB[m] = R((m & 1) == 1 ? 1 : 0);
  }
  auto degree = [&](const int l, R(&QW)[L1], const R(&QR)[L1]) {
    if (l > 0) {
      Gprev = Gl;
      Gl = Gl * g.w;
    }
    if (RANGED && (l < lo || l > hi)) {
      // outside the range: only the Legendre factors advance
      const Sc* __restrict__ bl = bA + l;
#pragma unroll
      for (int m = LMAX; m >= 0; --m)
        if (m <= l) QW[m] = g.c * QR[m] - bl[m * L1] * QW[m];
      return;
    }
    const Sc fl = Sc(l);
    const R dGl = fl * Gprev * g.om - (Sc(2) * fl + Sc(1)) * g.kap * Gl;
    R p[NW], dp[NW];
    p[0] = R(1);
    dp[0] = R(0);
    if constexpr (NMAXC >= 1) {
      p[1] = g.xi;
      dp[1] = R(1);
    }
    const Sc* __restrict__ bRl = bR + l * NW;
#pragma unroll
    for (int n = 2; n <= NMAXC; ++n) {
      const Sc b = bRl[n];
      p[n] = g.xi * p[n - 1] - b * p[n - 2];
      dp[n] = fma(g.xi, dp[n - 1], p[n - 1]) - b * dp[n - 2];
    }
    R psl = R(0), rhl = R(0), gxl = R(0), gyl = R(0), gzl = R(0);
    const Sc* __restrict__ Wl = W + l * l * NW;
    const Sc* __restrict__ bl = bA + l;             // bl[m L1] = b_{l,m}
    const Sc* __restrict__ kl = bA + L1 * L1 + l;   // kl[-m] = l - m
    // sigma = sum_n W_n p_n and its xi-derivative for one (l, j) row
    auto radial_sums = [&](const Sc* __restrict__ wc, R& sv, R& dv) {
      sv = R(wc[0]);
      dv = R(0);
      if constexpr (NMAXC >= 1) {
        sv = fma(wc[1], p[1], sv);
        dv = R(wc[1]);
      }
#pragma unroll
      for (int n = 2; n <= NMAXC; ++n) {
        sv = fma(wc[n], p[n], sv);
        dv = fma(wc[n], dp[n], dv);
      }
    };
    R Qup = R(0);  // Qt_l^(m+1)
#pragma unroll
    for (int m = LMAX; m >= 0; --m) {
      if (m <= l) {
        const R Q = g.c * QR[m] - bl[m * L1] * QW[m];
        QW[m] = Q;
        const R dQ = kl[-m] * Qup;
        Qup = Q;
        const Sc* __restrict__ wc = Wl + (m == 0 ? 0 : 2 * m - 1) * NW;
        R sc, dsc;
        radial_sums(wc, sc, dsc);
        if (m == 0) {
          psl = fma(Q, sc, psl);
          rhl = fma(Q, dsc, rhl);
          gzl = fma(dQ, sc, gzl);
        } else {
          R ss, dss;
          radial_sums(wc + NW, ss, dss);
          const R v1 = sc * Er[m] + ss * Ei[m];
          const R v2 = dsc * Er[m] + dss * Ei[m];
          const R v3 = sc * Er[m - 1] + ss * Ei[m - 1];
          const R v4 = ss * Er[m - 1] - sc * Ei[m - 1];
          const R mQ = Sc(m) * Q;
          psl = fma(Q, v1, psl);
          rhl = fma(Q, v2, rhl);
          gzl = fma(dQ, v1, gzl);
          gxl = fma(mQ, v3, gxl);
          gyl = fma(mQ, v4, gyl);
        }
      }
    }
    psi = fma(Gl, psl, psi);
    psir = fma(dGl, psl, fma(Gl * g.dxi, rhl, psir));
    gx = fma(Gl, gxl, gx);
    gy = fma(Gl, gyl, gy);
    gz = fma(Gl, gzl, gz);
  };
#pragma unroll 1
  for (int l = 0; l <= LMAX; l += 2) {
    degree(l, QA, QB);
    if (l + 1 <= LMAX) degree(l + 1, QB, QA);
  }
}

// a = -grad psi from psir and Gamma: grad psi = psi_r rhat + (1/r) (Gamma -
// (rhat . Gamma) rhat); zero at r = 0
template <typename R>
__device__ __forceinline__ void field_cartesian(const Geom<R>& g, const R psir, const R gx,
                                                const R gy, const R gz, R& axv, R& ayv, R& azv) {
  const R rg = g.ux * gx + g.uy * gy + g.c * gz;
  axv = R(0);
  ayv = R(0);
  azv = R(0);
  if (g.r > R(0)) {
    axv = -(psir * g.ux + g.ir * (gx - rg * g.ux));
    ayv = -(psir * g.uy + g.ir * (gy - rg * g.uy));
    azv = -(psir * g.c + g.ir * (gz - rg * g.c));
  }
}

template <typename R, int NMAXC, int LMAX>
__device__ __forceinline__ void field_eval(const R x, const R y, const R z,
                                           const scalar_t<R>* __restrict__ W,
                                           const scalar_t<R>* __restrict__ bR,
                                           const scalar_t<R>* __restrict__ bA, scalar_t<R> binv,
                                           scalar_t<R> alpha, scalar_t<R> inv_alpha, int amode,
                                           R& psi, R& axv, R& ayv, R& azv) {
  const Geom<R> g = make_geom<R>(x, y, z, R(binv), R(alpha), R(inv_alpha), amode);
  R psir, gx, gy, gz;
  field_sums<R, NMAXC, LMAX, false>(g, W, bR, bA, 0, LMAX, psi, psir, gx, gy, gz);
  field_cartesian<R>(g, psir, gx, gy, gz, axv, ayv, azv);
}

template <typename R, int MODE>
__device__ __forceinline__ void field_store(const ForceArgs<R>& a, const int64_t i, const R x,
                                            const R y, const R z, const R psi, R axv, R ayv, R azv,
                                            const R cx, const R cy, const R cz, const R gcx,
                                            const R gcy, const R gcz);

// Body of the field kernel: one particle per thread of a 256-thread block.
template <typename R, int NMAXC, int LMAX, int MODE, bool BATCHED>
__device__ __forceinline__ void field_body(const ForceArgs<R>& a) {
  int64_t i;
  const R* __restrict__ W = a.W;
  R cx = a.cx, cy = a.cy, cz = a.cz, gcx = a.gcx, gcy = a.gcy, gcz = a.gcz;
  if constexpr (BATCHED) {
    // every block lies inside one cluster: its id and tables are wave-uniform
    const int b = blockIdx.x;
    const int cl = __builtin_amdgcn_readfirstlane(a.blk_cluster[b]);
    const int64_t b0 = uniform_i64(a.blk_begin[b]), b1 = uniform_i64(a.blk_end[b]);
    i = b0 + threadIdx.x;
    if (i >= b1) return;
    W = a.W + (int64_t)cl * a.W_stride;
    const double* ct = a.centre_tab + 9 * (int64_t)cl;
    cx = R(uniform_f64(ct[0]));
    cy = R(uniform_f64(ct[1]));
    cz = R(uniform_f64(ct[2]));
    gcx = R(uniform_f64(ct[3]));
    gcy = R(uniform_f64(ct[4]));
    gcz = R(uniform_f64(ct[5]));
  } else {
    i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
  }
  const R x = a.x[i], y = a.y[i], z = a.z[i];
  R psi, axv, ayv, azv;
  field_eval<R, NMAXC, LMAX>(x, y, z, W, a.beta_rad, a.beta_ang, a.binv, a.alpha, a.inv_alpha,
                             a.amode, psi, axv, ayv, azv);
  field_store<R, MODE>(a, i, x, y, z, psi, axv, ayv, azv, cx, cy, cz, gcx, gcy, gcz);
}

// Field kernel body with each point's degrees split over S parts (for few
// particles: S times the waves, each with about 1/S of a point's work).  A
// 256-thread block takes P = 256/S particles; thread j works on particle
// j mod P and part j / P, which is uniform over a wave since P >= 64.  Part k
// sums degrees DegreeSplit::begin[k] .. begin[k+1]-1, the parts above 0 hand
// their partial sums to part 0 through LDS, and part 0 adds them and stores.
//
// The degree ranges minimise the largest part's cost, a degree costing
// 2l + 3 units (its Gegenbauer sweep and the radial sums of its 2l + 1 order
// columns, one unit being a sweep over n), with two more units charged to
// part 0 for the additions, the Cartesian transform and the stores.
template <int LMAX, int S>
struct DegreeSplit {
  int begin[S + 1] = {};
  static constexpr int cost(int b, int e) { return e * (e + 2) - b * (b + 2); }
  constexpr DegreeSplit() {
    constexpr int L1 = LMAX + 1;
    int best[S + 1][L1 + 1] = {};  // least largest cost of degrees [0, e) in k parts
    int cut[S + 1][L1 + 1] = {};
    for (int e = 0; e <= L1; ++e) best[1][e] = cost(0, e) + 2;
    for (int k = 2; k <= S; ++k)
      for (int e = 0; e <= L1; ++e) {
        best[k][e] = 1 << 30;
        for (int b = 0; b <= e; ++b) {
          const int v = best[k - 1][b] > cost(b, e) ? best[k - 1][b] : cost(b, e);
          if (v < best[k][e]) {
            best[k][e] = v;
            cut[k][e] = b;
          }
        }
      }
    begin[S] = L1;
    for (int k = S; k >= 1; --k) begin[k - 1] = k == 1 ? 0 : cut[k][begin[k]];
  }
};
template <typename R, int NMAXC, int LMAX, int MODE, int S>
__device__ __forceinline__ void field_body_split(const ForceArgs<R>& a) {
  static_assert(S >= 2 && 256 % S == 0 && 256 / S >= 64, "parts must be wave-uniform");
  constexpr int P = 256 / S;
  constexpr DegreeSplit<LMAX, S> sp{};
  __shared__ R part[S - 1][5][P];
  const int t = threadIdx.x % P;
  const int h = __builtin_amdgcn_readfirstlane(threadIdx.x / P);
  const int64_t i0 = (int64_t)blockIdx.x * P + t;
  const bool live = i0 < a.n;
  const int64_t i = live ? i0 : a.n - 1;  // every thread reaches the barrier
  const R x = a.x[i], y = a.y[i], z = a.z[i];
  const Geom<R> g = make_geom<R>(x, y, z, R(a.binv), R(a.alpha), R(a.inv_alpha), a.amode);
  int lo = sp.begin[0], hi = sp.begin[1] - 1;
#pragma unroll
  for (int k = 1; k < S; ++k)
    if (h == k) {
      lo = sp.begin[k];
      hi = sp.begin[k + 1] - 1;
    }
  R psi, psir, gx, gy, gz;
  field_sums<R, NMAXC, LMAX, true>(g, a.W, a.beta_rad, a.beta_ang, lo, hi, psi, psir, gx, gy, gz);
  if (h) {
    part[h - 1][0][t] = psi;
    part[h - 1][1][t] = psir;
    part[h - 1][2][t] = gx;
    part[h - 1][3][t] = gy;
    part[h - 1][4][t] = gz;
  }
  __syncthreads();
  if (!h) {
#pragma unroll
    for (int k = 0; k < S - 1; ++k) {
      psi += part[k][0][t];
      psir += part[k][1][t];
      gx += part[k][2][t];
      gy += part[k][3][t];
      gz += part[k][4][t];
    }
    R axv, ayv, azv;
    field_cartesian<R>(g, psir, gx, gy, gz, axv, ayv, azv);
    if (live)
      field_store<R, MODE>(a, i, x, y, z, psi, axv, ayv, azv, a.cx, a.cy, a.cz, a.gcx, a.gcy,
                           a.gcz);
  }
}

// Host tidal field and the stores of one particle: the forces (mode 0), the
// fused kick and drift (mode 1) or the adjoint accumulation (mode 2).
template <typename R, int MODE>
__device__ __forceinline__ void field_store(const ForceArgs<R>& a, const int64_t i, const R x,
                                            const R y, const R z, const R psi, R axv, R ayv, R azv,
                                            const R cx, const R cy, const R cz, const R gcx,
                                            const R gcy, const R gcz) {
  if (a.host.ncomp > 0) {
    R hx, hy, hz;
    host_grad<R>(a.host, cx + x, cy + y, cz + z, hx, hy, hz);
    axv += gcx - hx;
    ayv += gcy - hy;
    azv += gcz - hz;
  }
  if constexpr (MODE == 0) {
    a.ax[i] = axv;
    a.ay[i] = ayv;
    a.az[i] = azv;
    if (a.pot) a.pot[i] = psi;
  } else if constexpr (MODE == 1) {
    R vx = fma(a.kick, axv, a.vx[i]);
    R vy = fma(a.kick, ayv, a.vy[i]);
    R vz = fma(a.kick, azv, a.vz[i]);
    a.vx[i] = vx;
    a.vy[i] = vy;
    a.vz[i] = vz;
    if (a.ax) {  // null on the steps whose accelerations no later step reads
      a.ax[i] = axv;
      a.ay[i] = ayv;
      a.az[i] = azv;
    }
    if (a.drift != R(0) || a.xo != a.x) {
      a.xo[i] = fma(a.drift, vx, x);
      a.yo[i] = fma(a.drift, vy, y);
      a.zo[i] = fma(a.drift, vz, z);
    }
  } else {
    // adjoint: the coefficient part of a kick's vector-Jacobian product,
    // lambda_x += m a (a from the gamma-weighted coefficients), then the
    // reverse of the preceding drift, lambda_v += drift lambda_x
    const R mi = a.mass[i];
    const R lx = fma(mi, axv, a.ax[i]), ly = fma(mi, ayv, a.ay[i]), lz = fma(mi, azv, a.az[i]);
    a.ax[i] = lx;
    a.ay[i] = ly;
    a.az[i] = lz;
    if (a.drift != R(0)) {
      a.vx[i] = fma(a.drift, lx, a.vx[i]);
      a.vy[i] = fma(a.drift, ly, a.vy[i]);
      a.vz[i] = fma(a.drift, lz, a.vz[i]);
    }
  }
}

// Field kernel launch variants: the compiler's own register budget at the
// 256-thread block bound, or a budget for at least 4 (single) or 2 (double)
// waves per SIMD.  The autotuner picks.
template <typename R, int NMAXC, int LMAX, int MODE, bool BATCHED>
__global__ void __launch_bounds__(256) field_kernel(ForceArgs<R> a) {
  field_body<R, NMAXC, LMAX, MODE, BATCHED>(a);
}
template <typename R, int NMAXC, int LMAX, int MODE, bool BATCHED>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 4 : 2)))
field_kernel_o4(ForceArgs<R> a) {
  field_body<R, NMAXC, LMAX, MODE, BATCHED>(a);
}
template <typename R, int NMAXC, int LMAX, int MODE, int S>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 4 : 2)))
field_kernel_split(ForceArgs<R> a) {
  field_body_split<R, NMAXC, LMAX, MODE, S>(a);
}

// ---------------------------------------------------------------------------
// field pass on the matrix cores (single precision)
// ---------------------------------------------------------------------------
// Same sums as field_eval (Eq. total_potential and its gradient).  For one
// (l, m) the field needs four radial sums over n: sigma_c = sum_n W^c_n p_n,
// sigma_s likewise, and their xi-derivatives.  The derivative of the monic
// Gegenbauer basis is again a combination of that basis (from
// d C_n^lam / d xi = 2 lam C_{n-1}^(lam+1) = 2 sum_{k = n-1, n-3, ..} (k + lam)
// C_k^lam), d p_n / d xi = sum_k D_nk p_k, so the derivatives are sums over
// the same p_k with the coefficients W'_k = sum_n D_nk W_n.  The four sums of a
// wave's 64 particles are then one chain of 4x4x1 16-block FP32 MFMAs over n:
// the A operand is the coefficient quadruple (W^c, W'^c, W^s, W'^s)_n
// broadcast from one block, the B operand is each lane's own p_n, and row r of
// the product lands in result register r of that lane.  The quadruples live in
// LDS in register layout: for degree l, quadruple q = m NW + n is block q % 16
// (lanes 4 (q % 16) + r) of register q / 16, so an order group's operands are
// a few coalesced LDS reads per lane and every MFMA names its block as an
// immediate.  The Legendre recurrence, the radial recurrence and the angular
// combination stay on the VALU.  (On gfx950 the MFMA and VALU work of one SIMD
// does not co-execute here, so the kernel's time is about the sum of the two.)
typedef float mfma_f4 __attribute__((ext_vector_type(4)));

// orders whose accumulation chains one wave interleaves
constexpr int MFMA_GROUP = 2;

template <int NMAXC, int LMAX>
struct MfmaShape {
  static constexpr int L1 = LMAX + 1, NW = NMAXC + 1;
  // operand registers of degree l, and of the degrees below l
  static constexpr int nv(int l) { return ((l + 1) * NW + 15) / 16; }
  static constexpr int off(int l) {
    int s = 0;
    for (int k = 0; k < l; ++k) s += nv(k);
    return s;
  }
  static constexpr int IMG = off(L1) * 64;  // floats of the LDS operand image
  // radial recurrence constants b_n of each degree (rows of 4-float multiples)
  static constexpr int TS = (NW + 3) / 4 * 4;
  static constexpr int TAB = L1 * TS;
};

// Monic Legendre recurrence constant b_{l,m} (b_{m,m} = -1 starts order m).
__host__ __device__ constexpr double legendre_b(int l, int m) {
  return l == m ? -1.0
                : (l < m + 2 ? 0.0
                             : (l + m - 1.0) * (l - m - 1.0) / ((2.0 * l - 1.0) * (2.0 * l - 3.0)));
}

template <int Q>
__device__ __forceinline__ mfma_f4 mfma_bcast(const float a, const float b, const mfma_f4 c) {
  // CBSZ = 4: all 16 blocks take their A operand from block ABID = Q % 16
  return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 4, Q & 15, 0);
}

template <int I, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < E) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, E>(f);
  }
}
template <int I, int STEP, typename F>
__device__ __forceinline__ void static_for_down(F&& f) {
  if constexpr (I >= 0) {
    f(std::integral_constant<int, I>{});
    static_for_down<I - STEP, STEP>(f);
  }
}

// The LDS operand image of a block and the radial recurrence constants.  The
// image is zeroed first; then thread t < (LMAX + 1)^2 fills the quadruples of
// row t = (l, j) of the force weights W (rows n > nmax of W are zero): W_n,
// and the derivative coefficients W'_k = 2 (k + lam) kappa_k S_k from the
// suffix sums S_k = W_{k+1} / kappa_{k+1} + S_{k+2}, formed in double
// precision from the per-degree table dtab ([l][0][n] = 1 / kappa_n,
// [l][1][n] = 2 (n + lam) kappa_n).
template <int NMAXC, int LMAX>
__device__ __forceinline__ void build_mfma_operands(float* img, float* tab,
                                                    const float* __restrict__ W,
                                                    const double* __restrict__ dtab,
                                                    const float* __restrict__ bR) {
  using S = MfmaShape<NMAXC, LMAX>;
  constexpr int NW = S::NW;
  static_assert(S::IMG % 4 == 0, "operand image in float4 units");
  static_assert(S::L1 * S::L1 <= 256, "one thread of the 256-thread block per (l, j) row");
  for (int e = threadIdx.x; e < S::IMG / 4; e += blockDim.x)
    reinterpret_cast<float4*>(img)[e] = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int e = threadIdx.x; e < S::TAB; e += blockDim.x) {
    const int l = e / S::TS, n = e - l * S::TS;
    tab[e] = n < NW ? bR[l * NW + n] : 0.f;
  }
  __syncthreads();
  const int t = threadIdx.x;
  static_for<0, S::L1>([&](auto lc) {
    constexpr int l = decltype(lc)::value;
    if (t >= l * l && t < (l + 1) * (l + 1)) {
      const int j = t - l * l;
      const int m = (j + 1) >> 1;
      // j = 0 and odd j: cosine part (rows 0, 1); even j > 0: sine part (rows 2, 3)
      const int r0 = (j > 0 && (j & 1) == 0) ? 2 : 0;
      const float* __restrict__ Wr = W + t * NW;
      const double* __restrict__ ik = dtab + l * 2 * NW;
      const double* __restrict__ dk = ik + NW;
      float w[NW];
#pragma unroll
      for (int n = 0; n < NW; ++n) w[n] = Wr[n];
      float* dst = img + S::off(l) * 64 + r0;
      double s1 = 0.0, s2 = 0.0;  // S_{k+1}, S_{k+2}
#pragma unroll
      for (int k = NMAXC; k >= 0; --k) {
        const double v = k < NMAXC ? (double)w[k < NMAXC ? k + 1 : 0] * ik[k < NMAXC ? k + 1 : 0]
                                   : 0.0;
        const double sk = v + s2;
        s2 = s1;
        s1 = sk;
        const int q = m * NW + k;
        float* d = dst + (q >> 4) * 64 + 4 * (q & 15);
        d[0] = w[k];
        d[1] = (float)(dk[k] * sk);
      }
    }
  });
}

template <int NMAXC, int LMAX>
__device__ __noinline__ void build_mfma_operands_call(float* img, float* tab,
                                                      const float* __restrict__ W,
                                                      const double* __restrict__ dtab,
                                                      const float* __restrict__ bR) {
  build_mfma_operands<NMAXC, LMAX>(img, tab, W, dtab, bR);
}

// psi_SCF and a = -grad psi_SCF at one point per lane; every lane of the wave
// must be active (the MFMAs mix the lanes' operands).  Degrees and orders are
// compile-time sweeps, so one point's whole evaluation is straight-line code
// that the scheduler can interleave freely.
template <int NMAXC, int LMAX>
__device__ __forceinline__ void field_eval_mfma(const float x, const float y, const float z,
                                                const float* img, const float* tab,
                                                const float binv, const float alpha,
                                                const float inv_alpha, const int amode,
                                                float& psi, float& axv, float& ayv, float& azv) {
  using S = MfmaShape<NMAXC, LMAX>;
  constexpr int L1 = S::L1, NW = S::NW;
  const int lane = threadIdx.x & 63;
  Geom<float> g = make_geom<float>(x, y, z, binv, alpha, inv_alpha, amode);
  float Er[L1], Ei[L1];
  Er[0] = 1.f;
  Ei[0] = 0.f;
#pragma unroll
  for (int m = 1; m <= LMAX; ++m) {
    Er[m] = Er[m - 1] * g.ux - Ei[m - 1] * g.uy;
    Ei[m] = Er[m - 1] * g.uy + Ei[m - 1] * g.ux;
  }
  psi = 0.f;
  float psir = 0.f, gx = 0.f, gy = 0.f, gz = 0.f;
  float Gprev = 0.f, Gl = g.g0;
  // Legendre factors: the ping-pong arrays of the VALU pass (degree l writes
  // the array of its parity, reading the other one)
  float QA[L1], QB[L1];
#pragma unroll
  for (int m = 0; m <= LMAX; ++m) {
    QA[m] = (m & 1) == 0 ? 1.f : 0.f;
    QB[m] = (m & 1) == 1 ? 1.f : 0.f;
  }
  static_for<0, L1>([&](auto lc) {
    constexpr int l = decltype(lc)::value;
    float(&QW)[L1] = (l & 1) ? QB : QA;
    const float(&QR)[L1] = (l & 1) ? QA : QB;
    const float* src = img + S::off(l) * 64 + lane;
    const float* tl = tab + l * S::TS;
    if constexpr (l > 0) {
      Gprev = Gl;
      Gl = Gl * g.w;
    }
    const float dGl = float(l) * Gprev * g.om - float(2 * l + 1) * g.kap * Gl;
    float p[NW];
    p[0] = 1.f;
    if constexpr (NMAXC >= 1) p[1] = g.xi;
#pragma unroll
    for (int n = 2; n <= NMAXC; ++n) p[n] = g.xi * p[n - 1] - tl[n] * p[n - 2];
    float psl = 0.f, rhl = 0.f, gxl = 0.f, gyl = 0.f, gzl = 0.f;
    float Qup = 0.f;
    // (the first two degrees of an order, Qt_m^m = 1 and Qt_{m+1}^m = c, and
    // dQt_m^m = 0, are written out: a product with a zero operand is not
    // folded away under IEEE rules)
    auto legendre = [&](auto mc, float& Q, float& dQ) {
      constexpr int m = decltype(mc)::value;
      if constexpr (l == m)
        Q = 1.f;
      else if constexpr (l == m + 1)
        Q = g.c;
      else
        Q = g.c * QR[m] - float(legendre_b(l, m)) * QW[m];
      QW[m] = Q;
      if constexpr (l == m)
        dQ = 0.f;
      else
        dQ = float(l - m) * Qup;
      Qup = Q;
    };
    // The first order of a degree's sweep (m = l) starts its sums, and its dQ
    // is zero; E_0 = 1 gives the order-1 gradient terms directly.  (Products
    // with a zero or unit operand are not folded away under IEEE rules, so
    // these cases are written out.)
    auto combine = [&](auto mc, const float Q, const float dQ, const mfma_f4 acc) {
      constexpr int m = decltype(mc)::value;
      constexpr bool first = m == l;
      auto add = [&](float& sum, const float u, const float v) {
        if constexpr (first)
          sum = u * v;
        else
          sum = fmaf(u, v, sum);
      };
      const float sc = acc[0], dsc = acc[1];
      if constexpr (m == 0) {
        add(psl, Q, sc);
        add(rhl, Q, dsc);
        if constexpr (!first) gzl = fmaf(dQ, sc, gzl);
      } else {
        const float ss = acc[2], dss = acc[3];
        const float v1 = sc * Er[m] + ss * Ei[m];
        const float v2 = dsc * Er[m] + dss * Ei[m];
        float v3, v4;
        if constexpr (m == 1) {
          v3 = sc;
          v4 = ss;
        } else {
          v3 = sc * Er[m - 1] + ss * Ei[m - 1];
          v4 = ss * Er[m - 1] - sc * Ei[m - 1];
        }
        const float mQ = float(m) * Q;
        add(psl, Q, v1);
        add(rhl, Q, v2);
        if constexpr (!first) gzl = fmaf(dQ, v1, gzl);
        add(gxl, mQ, v3);
        add(gyl, mQ, v4);
      }
    };
    // the sums are due at each call: this keeps the compiler from holding
    // every group's accumulators until the end of the sweep
    auto sums_due = [&]() {
      asm volatile("" : "+v"(psl), "+v"(rhl), "+v"(gzl), "+v"(gxl), "+v"(gyl));
    };
    // orders from m = l down, in groups of up to MFMA_GROUP whose chains
    // interleave (independent accumulators hide the matrix-core latency)
    static_for_down<l, MFMA_GROUP>([&](auto mc) {
      constexpr int mt = decltype(mc)::value;  // top order of the group
      constexpr int gs = mt + 1 < MFMA_GROUP ? mt + 1 : MFMA_GROUP;
      // the operand registers this group's quadruples lie in, from LDS
      constexpr int vlo = ((mt - gs + 1) * NW) >> 4, vhi = (mt * NW + NMAXC) >> 4;
      float cw[vhi - vlo + 1];
#pragma unroll
      for (int v = vlo; v <= vhi; ++v) cw[v - vlo] = src[v * 64];
      float Q[gs], dQ[gs];
      mfma_f4 acc[gs];
      static_for<0, gs>([&](auto gc) {
        constexpr int k = decltype(gc)::value;
        legendre(std::integral_constant<int, mt - k>{}, Q[k], dQ[k]);
        acc[k] = mfma_f4{0.f, 0.f, 0.f, 0.f};
      });
      static_for<0, NW>([&](auto nc) {
        constexpr int n = decltype(nc)::value;
        static_for<0, gs>([&](auto gc) {
          constexpr int k = decltype(gc)::value;
          constexpr int q = (mt - k) * NW + n;
          acc[k] = mfma_bcast<q>(cw[(q >> 4) - vlo], p[n], acc[k]);
        });
      });
      static_for<0, gs>([&](auto gc) {
        constexpr int k = decltype(gc)::value;
        combine(std::integral_constant<int, mt - k>{}, Q[k], dQ[k], acc[k]);
      });
      sums_due();
    });
    if constexpr (l == 0) {
      // degree 0 starts the sums and has no angular gradient
      psi = Gl * psl;
      psir = fmaf(dGl, psl, (Gl * g.dxi) * rhl);
    } else {
      psi = fmaf(Gl, psl, psi);
      psir = fmaf(dGl, psl, fmaf(Gl * g.dxi, rhl, psir));
      if constexpr (l == 1) {
        gx = Gl * gxl;
        gy = Gl * gyl;
        gz = Gl * gzl;
      } else {
        gx = fmaf(Gl, gxl, gx);
        gy = fmaf(Gl, gyl, gy);
        gz = fmaf(Gl, gzl, gz);
      }
    }
    // likewise the degree's contribution
    asm volatile("" : "+v"(psi), "+v"(psir), "+v"(gx), "+v"(gy), "+v"(gz));
  });
  const float rg = g.ux * gx + g.uy * gy + g.c * gz;
  axv = 0.f;
  ayv = 0.f;
  azv = 0.f;
  if (g.r > 0.f) {
    axv = -(psir * g.ux + g.ir * (gx - rg * g.ux));
    ayv = -(psir * g.uy + g.ir * (gy - rg * g.uy));
    azv = -(psir * g.c + g.ir * (gz - rg * g.c));
  }
}

// Persistent blocks of 256 threads: each builds the operand image once, then
// takes the tiles of 256 particles blockIdx.x, blockIdx.x + gridDim.x, ...
// Lanes past the end evaluate the last particle (so that every lane joins the
// MFMAs) and store nothing.
template <int NMAXC, int LMAX, int MODE, bool INLINE_BUILD>
__device__ __forceinline__ void field_mfma_body(const ForceArgs<float>& a) {
  using S = MfmaShape<NMAXC, LMAX>;
  __shared__ __align__(16) float img[S::IMG];
  __shared__ float tab[S::TAB];
  if constexpr (INLINE_BUILD)
    build_mfma_operands<NMAXC, LMAX>(img, tab, a.W, a.dtab, a.beta_rad);
  else
    build_mfma_operands_call<NMAXC, LMAX>(img, tab, a.W, a.dtab, a.beta_rad);
  __syncthreads();
  const int64_t ntiles = (a.n + 255) / 256;
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t i = t * 256 + threadIdx.x;
    const bool live = i < a.n;
    const int64_t ic = live ? i : a.n - 1;
    const float x = a.x[ic], y = a.y[ic], z = a.z[ic];
    float psi, axv, ayv, azv;
    field_eval_mfma<NMAXC, LMAX>(x, y, z, img, tab, a.binv, a.alpha, a.inv_alpha, a.amode, psi,
                                 axv, ayv, azv);
    if (live)
      field_store<float, MODE>(a, i, x, y, z, psi, axv, ayv, azv, a.cx, a.cy, a.cz, a.gcx, a.gcy,
                               a.gcz);
  }
}

// Two register budgets: the compiler's own (the operand build is then a call,
// so that its registers do not add to the sweep's), and one for five waves
// per SIMD (which also keeps the accumulators in ordinary VGPRs).
template <int NMAXC, int LMAX, int MODE>
__global__ void __launch_bounds__(256) field_mfma_kernel(ForceArgs<float> a) {
  field_mfma_body<NMAXC, LMAX, MODE, false>(a);
}
template <int NMAXC, int LMAX, int MODE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5)))
field_mfma_kernel_o5(ForceArgs<float> a) {
  field_mfma_body<NMAXC, LMAX, MODE, true>(a);
}

// sum over the 64 lanes of a wave (every lane receives the total)
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Adjoint kernel of one kick at positions x_k with cotangent direction
// mu_i = c lambda_v,i (the Hessian-vector part of the vector-Jacobian product
// of the acceleration):
//   lambda_x,i += d/deps a(x_i + eps mu_i)
//              = -Hess psi_SCF(x_i) mu_i - Hess psi_host(R + x_i) mu_i,
// the SCF part by evaluating the field on dual numbers.  With a host, each
// block also writes the sums over its particles of -Hess psi_host(R + x_i) mu_i
// (3), mu_i (3) and -mu_i . d grad psi_host(R + x_i) / d p_ck (3 per
// component) to partials[block][0..31], in the order listed.
template <typename T, int NMAXC, int LMAX>
__global__ void __launch_bounds__(256) hvp_kernel(HvpArgs<T> a) {
  using D = Dual<T>;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = i < a.n;
  const int64_t ii = valid ? i : 0;
  const T x = a.x[ii], y = a.y[ii], z = a.z[ii];
  T mx = valid ? a.c * a.lvx[ii] : T(0);
  T my = valid ? a.c * a.lvy[ii] : T(0);
  T mz = valid ? a.c * a.lvz[ii] : T(0);
  D psi, ax, ay, az;
  field_eval<D, NMAXC, LMAX>(D(x, mx), D(y, my), D(z, mz), a.W, a.beta_rad, a.beta_ang, a.binv,
                             a.alpha, a.inv_alpha, a.amode, psi, ax, ay, az);
  T ox = ax.d, oy = ay.d, oz = az.d;
  if (a.host.ncomp > 0) {
    __shared__ T red[4][32];
    T v[32];
#pragma unroll
    for (int q = 0; q < 32; ++q) v[q] = T(0);
    const T px = a.cx + x, py = a.cy + y, pz = a.cz + z;
    T hx, hy, hz;
    host_hess_vec<T>(a.host, px, py, pz, mx, my, mz, hx, hy, hz);
    ox -= hx;
    oy -= hy;
    oz -= hz;
    if (valid) {
      v[0] = -hx;
      v[1] = -hy;
      v[2] = -hz;
      v[3] = mx;
      v[4] = my;
      v[5] = mz;
#pragma unroll
      for (int c = 0; c < kMaxHostComp; ++c)
        if (c < a.host.ncomp)
#pragma unroll
          for (int k = 0; k < 3; ++k)
            v[6 + 3 * c + k] = -host_dgrad_dparam_dot<T>(a.host, c, k, px, py, pz, mx, my, mz);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 32; ++q) {
      const T t = wave_sum(v[q]);
      if (lane == q) red[wave][q] = t;
    }
    __syncthreads();
    if (threadIdx.x < 32) {
      const int q = threadIdx.x;
      a.partials[(int64_t)blockIdx.x * 32 + q] = ((red[0][q] + red[1][q]) + red[2][q]) + red[3][q];
    }
  }
  if (valid) {
    a.lx[i] += ox;
    a.ly[i] += oy;
    a.lz[i] += oz;
  }
}

// ---------------------------------------------------------------------------
// Block coefficient kernel (single precision): the sums of Eq. (sumanlm) with
// four waves sharing each stage of P particles.
//   basis phase: one wave (wave k mod 4 at stage k) evaluates, one lane per
//     particle, xi and the angular-times-mass-radial-prefactor values
//     v_lj = m G_l Qt_l^m {Re, Im}(u^m) into the particle's LDS record, with
//     the recurrence constants folded in at compile time;
//   accumulation phase: every lane of the block owns one tile of NR rows (n)
//     x 4 columns of one degree l, rebuilds the radial column p_n^(l)(xi) from
//     p_0 = 1, p_1 = xi, and sweeps its group's share of the stage (group g
//     takes particles g, g + G, ...), reading its four columns with one
//     128-bit LDS load;
//   folds: every FOLD stages (and at the end of the unit) the G groups'
//     tiles are summed pairwise through LDS and the result is added to the
//     unit's (hi, lo) pair of partial rows with an error-free two-sum, so the
//     single-precision sums run over at most FOLD * P / G particles whatever N
//     is, and the rounding error of each fold is carried in lo.  The same
//     kernel in double precision (a variant of the double-precision plans)
//     adds its folds into one partial row per unit, and its records take two
//     128-bit loads per tile.
// The l-block of a record holds [Re_0, 0, Re_1, Im_1, .., Re_l, Im_l] padded
// with zeros to a multiple of 4 (so the sine-cosine pairs are 8-byte aligned
// for 64-bit stores); the record stride PS is a multiple of 4 with PS/4 odd,
// which keeps the bank conflicts of the 128-bit tile loads low (an even PS/4
// measured three times the conflict cycles).
// ---------------------------------------------------------------------------
// Order units of the block kernel's basis phase: order 0, order 1, the pairs
// (2k, 2k+1) for k >= 1, and order lmax alone when it is even and >= 2.  A
// unit writes whole 4-column chunks of the records (order 0 and order 1 write
// the two halves of chunk 0), so every record slot is rewritten each stage.
// The units are assigned to the four waves at compile time, largest first to
// the least-loaded wave (cost = number of (l, m) values).
template <int LMAX>
struct OrderUnits {
  static constexpr int NPAIR = LMAX >= 3 ? (LMAX - 1) / 2 : 0;          // pairs k = 1..NPAIR
  static constexpr bool SINGLE = LMAX >= 2 && LMAX % 2 == 0;
  static constexpr int NU = (LMAX >= 1 ? 2 : 1) + NPAIR + (SINGLE ? 1 : 0);
  // kind: 0 = order 0, 1 = order 1, 2 = pair (ma, ma + 1), 3 = order ma alone
  static constexpr int kind(int u) {
    return u == 0 ? 0 : (LMAX >= 1 && u == 1 ? 1 : (u < NU - (SINGLE ? 1 : 0) ? 2 : 3));
  }
  static constexpr int ma(int u) {
    return kind(u) == 0 ? 0 : kind(u) == 1 ? 1 : kind(u) == 2 ? 2 * (u - 1) : LMAX;
  }
  static constexpr int cost(int u) {
    return kind(u) == 2 ? (LMAX - ma(u) + 1) + (LMAX - ma(u)) : (LMAX - ma(u) + 1);
  }
  // wave (of WS sharing a slab of particles) that evaluates unit uq
  static constexpr int owner(int uq, int WS) {
    int load[4] = {0, 0, 0, 0};
    bool done[NU > 0 ? NU : 1] = {};
    int own = 0;
    for (int it = 0; it < NU; ++it) {
      int best = -1;
      for (int u = 0; u < NU; ++u)
        if (!done[u] && (best < 0 || cost(u) > cost(best))) best = u;
      int w = 0;
      for (int q = 1; q < WS; ++q)
        if (load[q] < load[w]) w = q;
      load[w] += cost(best);
      done[best] = true;
      if (best == uq) own = w;
    }
    return own;
  }
};

// u^M (complex) and w^M (real) by squaring, at compile time over M.
template <int M, typename R>
__device__ __forceinline__ void cpow_u(R ux, R uy, R& er, R& ei) {
  if constexpr (M == 0) {
    er = R(1);
    ei = R(0);
  } else if constexpr (M == 1) {
    er = ux;
    ei = uy;
  } else if constexpr (M % 2 == 0) {
    R hr, hi;
    cpow_u<M / 2>(ux, uy, hr, hi);
    er = hr * hr - hi * hi;
    ei = R(2) * hr * hi;
  } else {
    R hr, hi;
    cpow_u<M - 1>(ux, uy, hr, hi);
    er = hr * ux - hi * uy;
    ei = hr * uy + hi * ux;
  }
}
template <int M, typename R>
__device__ __forceinline__ R rpow(R w) {
  if constexpr (M == 0) return R(1);
  else if constexpr (M == 1) return w;
  else if constexpr (M % 2 == 0) {
    const R h = rpow<M / 2>(w);
    return h * h;
  } else {
    return rpow<M - 1>(w) * w;
  }
}

// Monic Legendre factor Qt_l^m from the two previous degrees (Qt_m^m = 1,
// Qt_{m+1}^m = c); in single precision, order 0, whose even degrees carry a
// constant term, takes its recurrence constants as float pairs (hi + lo) so
// that their rounding leaves no bias in an isotropic average.
template <int L, int M, typename R>
__device__ __forceinline__ R legendre_next(R c, R Q1, R Q0) {
  if constexpr (L == M) {
    return R(1);
  } else if constexpr (L == M + 1) {
    return c;
  } else if constexpr (M == 0 && sizeof(R) == 4) {
    constexpr double gd = legendre_b(L, M);
    constexpr float ghi = float(gd);
    constexpr float glo = float(gd - double(ghi));
    return fmaf(-glo, Q0, c * Q1 - ghi * Q0);
  } else {
    constexpr R gam = R(legendre_b(L, M));
    return c * Q1 - gam * Q0;
  }
}

// record stores of 2 and 4 consecutive values (16- and 8-byte aligned slots
// in single precision; two 16-byte stores for four doubles)
__device__ __forceinline__ void store2(float* d, float a, float b) {
  *reinterpret_cast<float2*>(d) = make_float2(a, b);
}
__device__ __forceinline__ void store4(float* d, float a, float b, float c, float e) {
  *reinterpret_cast<float4*>(d) = make_float4(a, b, c, e);
}
__device__ __forceinline__ void store2(double* d, double a, double b) {
  *reinterpret_cast<double2*>(d) = make_double2(a, b);
}
__device__ __forceinline__ void store4(double* d, double a, double b, double c, double e) {
  *reinterpret_cast<double2*>(d) = make_double2(a, b);
  *reinterpret_cast<double2*>(d + 2) = make_double2(c, e);
}

// The values of one order unit for one particle into its record r:
// m G_l Qt_l^m {Re, Im}(u^m), with mg0 = m G_0 (zero for a padding particle).
template <int LMAX, int U, typename R, typename AoffF>
__device__ __forceinline__ void basis_unit(R* r, const Geom<R>& g, R mg0, AoffF aoff) {
  using OU = OrderUnits<LMAX>;
  constexpr int K = OU::kind(U), MA = OU::ma(U);
  R era, eia, erb = R(0), eib = R(0);
  cpow_u<MA>(g.ux, g.uy, era, eia);
  if constexpr (K == 2) {
    erb = era * g.ux - eia * g.uy;
    eib = era * g.uy + eia * g.ux;
  }
  R G = mg0 * rpow<MA>(g.w);  // m G_l at l = MA
  R Qa0 = R(0), Qa1 = R(0), Qb0 = R(0), Qb1 = R(0);
  static_for<MA, LMAX + 1>([&](auto lc) {
    constexpr int l = decltype(lc)::value;
    const R Qa = legendre_next<l, MA>(g.c, Qa1, Qa0);
    Qa0 = Qa1;
    Qa1 = Qa;
    const R va = Qa * G;
    R* d = r + aoff(l);
    if constexpr (K == 0) {
      if constexpr (l == 0)
        store4(d, va, R(0), R(0), R(0));
      else
        store2(d, va, R(0));
    } else if constexpr (K == 1) {
      store2(d + 2, va * era, va * eia);
    } else if constexpr (K == 2) {
      R vb = R(0);
      if constexpr (l >= MA + 1) {
        const R Qb = legendre_next<l, MA + 1>(g.c, Qb1, Qb0);
        Qb0 = Qb1;
        Qb1 = Qb;
        vb = Qb * G;
      }
      store4(d + 2 * MA, va * era, va * eia, vb * erb, vb * eib);
    } else {
      store4(d + 2 * MA, va * era, va * eia, R(0), R(0));
    }
    if constexpr (l < LMAX) G *= g.w;
  });
}

template <int LMAX, int WS, int W, typename R, typename AoffF>
__device__ __forceinline__ void basis_wave(R* r, const Geom<R>& g, R mg0, AoffF aoff) {
  using OU = OrderUnits<LMAX>;
  static_for<0, OU::NU>([&](auto uc) {
    constexpr int u = decltype(uc)::value;
    if constexpr (OU::owner(u, WS) == W) basis_unit<LMAX, u>(r, g, mg0, aoff);
  });
}

template <int NMAXC, int LMAX, typename R = float>
struct BlkShape {
  static constexpr int JT = 4;
  static constexpr int NR = NMAXC + 1;
  static constexpr int NT = ntiles_c(LMAX, JT);
  static constexpr int THREADS = 256;
  static constexpr int AL = JT * NT;  // angular slots per record
  static constexpr int XI = AL;       // slot of xi
  static constexpr int PS = ((AL / 4 + 1) % 2 == 1) ? (AL / 4 + 1) * 4 : (AL / 4 + 2) * 4;
  // a stage holds SLABS slabs of up to 64 particles (one particle per lane in
  // the basis phase): the most (1, 2 or 4) whose records fit 39 KB (single
  // precision: four blocks share a compute unit's LDS) or 78 KB (double: two)
  static constexpr int RB = (int)sizeof(R);
  static constexpr int LDS_REC = (RB == 4 ? 39 : 78) * 1024 - RB * (LMAX + 1) * NR;
  static constexpr int SLABS =
      (4 * 64 * PS * RB <= LDS_REC) ? 4 : ((2 * 64 * PS * RB <= LDS_REC) ? 2 : 1);
  static constexpr int WS = 4 / SLABS;  // waves sharing a slab (they split its order units)
  static constexpr int G = (THREADS / NT) > 64 ? 64 : (THREADS / NT);
  static constexpr int PPG = (64 * SLABS) / G;  // particles per group and stage
  static constexpr int P = G * PPG;             // particles per stage
  static constexpr int SLOT = NT * NR * JT;   // values of one group's tiles
  static constexpr int NSLOT = (P * PS) / SLOT;  // group tiles the stage buffer holds
  static constexpr int aoff(int l) { return JT * ntiles_c(l - 1, JT); }
  static_assert(G >= 1 && NT * G <= THREADS, "tiles must fit the block");
  static_assert(NSLOT >= 1, "the stage buffer must hold one group's tiles");
};

// waves per SIMD the block kernel is compiled for: single precision 4 (at
// most 128 registers) when its tiles have at most 17 rows, else 3; double
// precision 2
template <int NMAXC, typename R>
constexpr int blk_waves() { return sizeof(R) == 8 ? 2 : (NMAXC <= 16 ? 4 : 3); }

// four consecutive record values (one 16-byte load in single precision, two
// in double)
__device__ __forceinline__ void load4(const float* p, float (&v)[4]) {
  const float4 q = *reinterpret_cast<const float4*>(p);
  v[0] = q.x;
  v[1] = q.y;
  v[2] = q.z;
  v[3] = q.w;
}
__device__ __forceinline__ void load4(const double* p, double (&v)[4]) {
  const double2 q0 = *reinterpret_cast<const double2*>(p);
  const double2 q1 = *reinterpret_cast<const double2*>(p + 2);
  v[0] = q0.x;
  v[1] = q0.y;
  v[2] = q1.x;
  v[3] = q1.y;
}
__device__ __forceinline__ float fma_r(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fma_r(double a, double b, double c) { return fma(a, b, c); }

// Block coefficient kernel.  R = float is the single-precision pass with
// compensated folds into (hi, lo) rows; R = double (a variant of the
// double-precision plans) adds its folds into one double row per unit.
template <int NMAXC, int LMAX, int FOLD, typename R = float>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(blk_waves<NMAXC, R>(), blk_waves<NMAXC, R>())))
coef_blk_kernel(CoefArgs<R> a) {
  using S = BlkShape<NMAXC, LMAX, R>;
  constexpr int NR = S::NR, NT = S::NT, G = S::G, P = S::P, PS = S::PS, XI = S::XI;
  constexpr int PPG = S::PPG, SLOT = S::SLOT, NSLOT = S::NSLOT, L2 = (LMAX + 1) * (LMAX + 1);
  __shared__ __align__(16) R rec[P * PS];

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int grp = tid / NT, tau = tid % NT;
  const bool tv = grp < G;
  // degree and first column of this lane's tile
  int tl = 0, tc = 0;
  {
    int rem = tau;
#pragma unroll
    for (int ll = 0; ll <= LMAX; ++ll) {
      const int nt = (2 * ll + 1 + 3) / 4;
      if (rem >= 0 && rem < nt) {
        tl = ll;
        tc = 4 * rem;
      }
      rem -= nt;
    }
  }
  // radial recurrence constants of every degree, read per stage from LDS so
  // that they are not live through the basis phase
  __shared__ __align__(16) R btab[(LMAX + 1) * NR];
  for (int i = tid; i < (LMAX + 1) * NR; i += 256) btab[i] = a.beta_rad[i];

  // particle range and partial-row pair of this unit
  const int unit = blockIdx.x;
  int64_t begin, end;
  int slot;
  if (a.seg_begin) {
    begin = a.seg_begin[unit];
    end = a.seg_end[unit];
    slot = a.seg_slot[unit];
  } else {
    begin = a.begin + (a.stages * unit / a.nunits) * P;
    end = a.begin + (a.stages * (unit + 1) / a.nunits) * P;
    if (end > a.n) end = a.n;
    slot = unit;
  }
  if (begin >= end) return;  // (uniform over the block; launches give every unit a stage)

  // Wave w works on slab w / WS of each stage and evaluates the order units
  // of rank sub = w mod WS; its lane holds particle q = 64 slab + lane of the
  // current stage (loaded one stage ahead).  Loads are unconditional, from an
  // index clamped into the unit's range; pw (0 or 1) removes the particles
  // past the range.
  constexpr int WS = S::WS;
  const int sub = wave % WS, q = (wave / WS) * 64 + lane;
  R px, py, pz, pm, pw;
  {
    const int64_t gi0 = begin + q;
    const bool ok = q < P && gi0 < end;
    const int64_t gi = ok ? gi0 : end - 1;
    px = a.x[gi];
    py = a.y[gi];
    pz = a.z[gi];
    pm = a.m[gi];
    pw = ok ? R(1) : R(0);
  }
  __syncthreads();

  R acc[NR][4];
#pragma unroll
  for (int n = 0; n < NR; ++n)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[n][j] = R(0);

  R* hi = a.partials + (int64_t)slot * (a.one_row ? 1 : 2) * a.T;
  [[maybe_unused]] R* lo = hi + a.T;  // (single precision; unused when one_row)
  bool first_fold = true;
  int k = 0, since = 0;
  for (int64_t base = begin; base < end; base += P, ++k) {
    // ---- basis phase: every wave evaluates the geometry of the stage's
    // particles and the values of its own order units ------------------------
    if (q < P) {
      R* r = rec + q * PS;
      const Geom<R> g = make_geom<R>(px, py, pz, a.binv, a.alpha, a.inv_alpha, a.amode);
      if (sub == 0) r[XI] = g.xi;
      const R mg0 = (pm * pw) * g.g0;
      auto aoff = [](int l) { return S::aoff(l); };
      if constexpr (WS == 1) {
        basis_wave<LMAX, 1, 0>(r, g, mg0, aoff);
      } else if constexpr (WS == 2) {
        if (sub == 0) basis_wave<LMAX, 2, 0>(r, g, mg0, aoff);
        else basis_wave<LMAX, 2, 1>(r, g, mg0, aoff);
      } else {
        switch (sub) {
          case 0: basis_wave<LMAX, 4, 0>(r, g, mg0, aoff); break;
          case 1: basis_wave<LMAX, 4, 1>(r, g, mg0, aoff); break;
          case 2: basis_wave<LMAX, 4, 2>(r, g, mg0, aoff); break;
          default: basis_wave<LMAX, 4, 3>(r, g, mg0, aoff); break;
        }
      }
    }
    {
      // particle of the next stage; the barriers below wait for LDS traffic
      // only, so the load stays in flight through the accumulation phase
      const int64_t gi0 = base + (int64_t)P + q;
      const bool ok = q < P && gi0 < end;
      const int64_t gi = ok ? gi0 : end - 1;
      px = a.x[gi];
      py = a.y[gi];
      pz = a.z[gi];
      pm = a.m[gi];
      pw = ok ? R(1) : R(0);
    }
    __syncthreads();
    // ---- accumulation phase -----------------------------------------------
    if (tv) {
      R bl[NR];
#pragma unroll
      for (int n = 2; n < NR; ++n) bl[n] = btab[tl * NR + n];
      const R* rp = rec + grp * PS;
#pragma unroll 1
      for (int ii = 0; ii < PPG; ++ii) {
        R a4[4];
        load4(rp + 4 * tau, a4);
        const R xi = rp[XI];
        rp += G * PS;
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[0][j] += a4[j];
        if constexpr (NR > 1) {
          R p0 = R(1), p1 = xi;
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[1][j] = fma_r(p1, a4[j], acc[1][j]);
#pragma unroll
          for (int n = 2; n < NR; ++n) {
            const R p2 = n == 2 ? fma_r(xi, p1, -bl[2]) : fma_r(xi, p1, -bl[n] * p0);
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[n][j] = fma_r(p2, a4[j], acc[n][j]);
            p0 = p1;
            p1 = p2;
          }
        }
      }
    }
    ++since;
    const bool last = base + P >= end;
    if (since == FOLD || last) {
      __syncthreads();  // every group has finished reading the stage
      // ---- groups summed pairwise into group 0 through the stage buffer ----
      for (int active = G; active > 1;) {
        const int half = (active + 1) / 2, movers = active - half;
        for (int c0 = 0; c0 < movers; c0 += NSLOT) {
          const int c1 = movers < c0 + NSLOT ? movers : c0 + NSLOT;
          if (tv && grp >= half + c0 && grp < half + c1) {
            R* d = rec + (grp - half - c0) * SLOT + tau * NR * 4;
#pragma unroll
            for (int n = 0; n < NR; ++n) store4(d + 4 * n, acc[n][0], acc[n][1], acc[n][2], acc[n][3]);
          }
          __syncthreads();
          if (tv && grp >= c0 && grp < c1) {
            const R* s = rec + (grp - c0) * SLOT + tau * NR * 4;
#pragma unroll
            for (int n = 0; n < NR; ++n) {
              R v[4];
              load4(s + 4 * n, v);
              acc[n][0] += v[0];
              acc[n][1] += v[1];
              acc[n][2] += v[2];
              acc[n][3] += v[3];
            }
          }
          __syncthreads();
        }
        active = half;
      }
      // ---- two-sum fold of the block's sums into the unit's (hi, lo) rows ----
      // group 0 leaves its tiles in the stage buffer; every thread then folds
      // coefficients t = tid, tid + 256, .. (coalesced rows)
      if (tv && grp == 0) {
        R* d = rec + tau * NR * 4;
#pragma unroll
        for (int n = 0; n < NR; ++n) store4(d + 4 * n, acc[n][0], acc[n][1], acc[n][2], acc[n][3]);
      }
      __syncthreads();
      for (int t = tid; t < a.T; t += 256) {
        const int n = t / L2, lj = t - n * L2;
        const int l = (int)sqrtf((float)lj + 0.5f), j = lj - l * l;
        // column of j in the l-block, and the tile holding it
        const int c = j == 0 ? 0 : j + 1;
        const int tau_t = (l == 0 ? 0 : l + (l - 1) * (l - 1) / 4) + (c >> 2);
        const R v = rec[(tau_t * NR + n) * 4 + (c & 3)];
        if (first_fold) {
          hi[t] = v;
          if constexpr (sizeof(R) == 4)
            if (!a.one_row) lo[t] = 0.f;
        } else if constexpr (sizeof(R) == 4) {
          const float h = hi[t];
          const float sum = h + v;
          const float bp = sum - h;
          const float err = (h - (sum - bp)) + (v - bp);
          hi[t] = sum;
          lo[t] = lo[t] + err;
        } else {
          hi[t] = hi[t] + v;  // double precision: one row, plain sums
        }
      }
#pragma unroll
      for (int n = 0; n < NR; ++n)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[n][j] = R(0);
      first_fold = false;
      since = 0;

    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// engines
// ---------------------------------------------------------------------------
template <typename R>
struct CoefVariants;
template <>
struct CoefVariants<float> {
  static constexpr int N = 3;
  static constexpr int LPP[N] = {2, 1, 4};
  static constexpr int WPB[N] = {1, 1, 1};
};
template <>
struct CoefVariants<double> {
  static constexpr int N = 3;
  static constexpr int LPP[N] = {4, 2, 8};
  static constexpr int WPB[N] = {1, 1, 1};
};

// stages per fold of the single-precision block coefficient kernel
constexpr int kCoefFold = 16;

template <typename R, int NMAXC, int LMAX>
struct EngineImpl final : Engine {
  using V = CoefVariants<R>;
  // Single-precision plans have one coefficient kernel, the block kernel with
  // compensated folds; double-precision plans have the V::N wave-unit variants
  // and the block kernel as variant V::N.
  static constexpr bool kBlk = sizeof(R) == 4;
  using BS = BlkShape<NMAXC, LMAX, R>;
  static bool is_blk(int v) { return kBlk || v == V::N; }
  int nmaxc() const override { return NMAXC; }
  int lmax() const override { return LMAX; }
  int dtype() const override { return sizeof(R) == 4 ? 0 : 1; }
  size_t real_size() const override { return sizeof(R); }
  int coef_variants() const override { return kBlk ? 1 : V::N + 1; }
  int stage_particles(int v) const override { return is_blk(v) ? BS::P : 64 / V::LPP[v]; }
  int fold_stages(int v) const override {
    (void)v;
    return is_blk(v) ? kCoefFold : 0;
  }
  int rows_per_unit(int v) const override {
    if (kBlk) return 2;     // the (hi, lo) pair
    if (v == V::N) return 1;  // double block kernel: one row
    return v == 0 ? rows_t<V::LPP[0]>() : v == 1 ? rows_t<V::LPP[1]>() : rows_t<V::LPP[2]>();
  }
  template <int LPP>
  static constexpr int rows_t() {
    using S = CoefShape<R, NMAXC, LMAX, LPP>;
    return (S::G == 1 || S::NT * S::NR * S::JT <= S::P * S::PS) ? 1 : S::G;
  }
  int max_resident_units(int v) const override {
    int per_cu = 0;
    hipError_t e;
    if (is_blk(v)) {
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, coef_blk_kernel<NMAXC, LMAX, kCoefFold, R>, 256, 0);
      if (e != hipSuccess || per_cu <= 0) per_cu = 1;
      return per_cu;  // a unit is a block of four waves
    } else if constexpr (!kBlk) {
      if (v == 0)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, coef_kernel<R, NMAXC, LMAX, V::LPP[0], V::WPB[0]>, 64 * V::WPB[0], 0);
      else if (v == 1)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, coef_kernel<R, NMAXC, LMAX, V::LPP[1], V::WPB[1]>, 64 * V::WPB[1], 0);
      else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, coef_kernel<R, NMAXC, LMAX, V::LPP[2], V::WPB[2]>, 64 * V::WPB[2], 0);
      if (e != hipSuccess || per_cu <= 0) per_cu = 1;
      return per_cu * V::WPB[v];
    }
    return 1;
  }
  hipError_t launch_coef(const void* args, int nunits, int v, hipStream_t s) const override {
    if (nunits <= 0) return hipSuccess;
    const CoefArgs<R>& ca = *(const CoefArgs<R>*)args;
    if (is_blk(v)) {
      coef_blk_kernel<NMAXC, LMAX, kCoefFold, R><<<nunits, 256, 0, s>>>(ca);
    } else if constexpr (!kBlk) {
      const int wpb = V::WPB[v];
      const int nblocks = (nunits + wpb - 1) / wpb;
      if (v == 0)
        coef_kernel<R, NMAXC, LMAX, V::LPP[0], V::WPB[0]><<<nblocks, 64 * V::WPB[0], 0, s>>>(ca);
      else if (v == 1)
        coef_kernel<R, NMAXC, LMAX, V::LPP[1], V::WPB[1]><<<nblocks, 64 * V::WPB[1], 0, s>>>(ca);
      else
        coef_kernel<R, NMAXC, LMAX, V::LPP[2], V::WPB[2]><<<nblocks, 64 * V::WPB[2], 0, s>>>(ca);
    }
    return hipGetLastError();
  }
  // field variants: 0 and 1 = VALU kernel under two register budgets; 2 and 3
  // (single precision) = matrix-core kernel under two register budgets; the
  // last two (4 and 5 in single, 2 and 3 in double precision) = VALU kernel
  // with each point's degrees split over 2 or 4 waves.  The batched step runs
  // variant 1's kernel for variants 1 to 3; the adjoint's accumulation pass
  // runs variant 0's for variants 0 to 3 and the split kernels for theirs.
  int field_variants() const override { return sizeof(R) == 4 ? 6 : 4; }
  // the first split variant (two parts; the next one has four)
  static constexpr int kSplitVariant = sizeof(R) == 4 ? 4 : 2;
  // resident blocks of a persistent kernel on the device
  template <typename K>
  static int64_t resident_blocks(K kernel) {
    int per_cu = 0, dev = 0, ncu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0) != hipSuccess ||
        per_cu <= 0)
      per_cu = 1;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        ncu <= 0)
      ncu = 1;
    return (int64_t)per_cu * ncu;
  }
  hipError_t launch_force(const void* args, int64_t nblocks, int mode, int fv,
                          hipStream_t s) const override {
    if (nblocks <= 0) return hipSuccess;
    const ForceArgs<R>& fa = *(const ForceArgs<R>*)args;
    if constexpr (sizeof(R) == 4) {
      if ((fv == 2 || fv == 3) && mode != 2 && !fa.blk_cluster) {
        // nblocks tiles of 256 particles over at most one resident round of blocks
        static const int64_t cap[2] = {resident_blocks(field_mfma_kernel<NMAXC, LMAX, 1>),
                                       resident_blocks(field_mfma_kernel_o5<NMAXC, LMAX, 1>)};
        const dim3 g((unsigned)(nblocks < cap[fv - 2] ? nblocks : cap[fv - 2]));
        if (fv == 2) {
          if (mode == 0)
            field_mfma_kernel<NMAXC, LMAX, 0><<<g, 256, 0, s>>>(fa);
          else
            field_mfma_kernel<NMAXC, LMAX, 1><<<g, 256, 0, s>>>(fa);
        } else {
          if (mode == 0)
            field_mfma_kernel_o5<NMAXC, LMAX, 0><<<g, 256, 0, s>>>(fa);
          else
            field_mfma_kernel_o5<NMAXC, LMAX, 1><<<g, 256, 0, s>>>(fa);
        }
        return hipGetLastError();
      }
    }
    const dim3 g((unsigned)nblocks);
    if (fv >= kSplitVariant && !fa.blk_cluster) {
      // 128 (two parts) or 64 (four parts) particles a block
      const int64_t per = fv == kSplitVariant ? 128 : 64;
      const dim3 gs((unsigned)((fa.n + per - 1) / per));
      if (fv == kSplitVariant) {
        if (mode == 0)
          field_kernel_split<R, NMAXC, LMAX, 0, 2><<<gs, 256, 0, s>>>(fa);
        else if (mode == 1)
          field_kernel_split<R, NMAXC, LMAX, 1, 2><<<gs, 256, 0, s>>>(fa);
        else
          field_kernel_split<R, NMAXC, LMAX, 2, 2><<<gs, 256, 0, s>>>(fa);
      } else {
        if (mode == 0)
          field_kernel_split<R, NMAXC, LMAX, 0, 4><<<gs, 256, 0, s>>>(fa);
        else if (mode == 1)
          field_kernel_split<R, NMAXC, LMAX, 1, 4><<<gs, 256, 0, s>>>(fa);
        else
          field_kernel_split<R, NMAXC, LMAX, 2, 4><<<gs, 256, 0, s>>>(fa);
      }
      return hipGetLastError();
    }
    if (fv >= 1 && mode != 2) {
      if (fa.blk_cluster)
        field_kernel_o4<R, NMAXC, LMAX, 1, true><<<g, 256, 0, s>>>(fa);
      else if (mode == 0)
        field_kernel_o4<R, NMAXC, LMAX, 0, false><<<g, 256, 0, s>>>(fa);
      else
        field_kernel_o4<R, NMAXC, LMAX, 1, false><<<g, 256, 0, s>>>(fa);
    } else {
      if (fa.blk_cluster)
        field_kernel<R, NMAXC, LMAX, 1, true><<<g, 256, 0, s>>>(fa);
      else if (mode == 0)
        field_kernel<R, NMAXC, LMAX, 0, false><<<g, 256, 0, s>>>(fa);
      else if (mode == 1)
        field_kernel<R, NMAXC, LMAX, 1, false><<<g, 256, 0, s>>>(fa);
      else
        field_kernel<R, NMAXC, LMAX, 2, false><<<g, 256, 0, s>>>(fa);
    }
    return hipGetLastError();
  }
  // adjoint gamma pass: variant 0's lane split on dual numbers
  using GS = CoefShape<Dual<R>, NMAXC, LMAX, V::LPP[0]>;
  int gamma_stage_particles() const override { return GS::P; }
  int gamma_rows_per_unit() const override {
    return (GS::G == 1 || GS::NT * GS::NR * GS::JT <= GS::P * GS::PS) ? 1 : GS::G;
  }
  int gamma_resident_units() const override {
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, coef_kernel<Dual<R>, NMAXC, LMAX, V::LPP[0], 1>, 64, 0);
    if (e != hipSuccess || per_cu <= 0) per_cu = 1;
    return per_cu;
  }
  hipError_t launch_gamma(const void* args, int nunits, hipStream_t s) const override {
    if (nunits <= 0) return hipSuccess;
    const CoefArgs<Dual<R>>& ca = *(const CoefArgs<Dual<R>>*)args;
    coef_kernel<Dual<R>, NMAXC, LMAX, V::LPP[0], 1><<<nunits, 64, 0, s>>>(ca);
    return hipGetLastError();
  }
  hipError_t launch_hvp(const void* args, int64_t nblocks, hipStream_t s) const override {
    if (nblocks <= 0) return hipSuccess;
    const HvpArgs<R>& ha = *(const HvpArgs<R>*)args;
    hvp_kernel<R, NMAXC, LMAX><<<dim3((unsigned)nblocks), 256, 0, s>>>(ha);
    return hipGetLastError();
  }
  const char* describe() const override {
    static char buf[200];
    if constexpr (kBlk) {
      snprintf(buf, sizeof(buf),
               "f32 nmax<=%d lmax=%d coef: block kernel, %d x %d tiles, %d groups, %d particles "
               "per stage, two-sum folds every %d stages",
               NMAXC, LMAX, BS::NR, BS::JT, BS::G, BS::P, kCoefFold);
    } else {
      using S0 = CoefShape<R, NMAXC, LMAX, V::LPP[0]>;
      using S2 = CoefShape<R, NMAXC, LMAX, V::LPP[2]>;
      snprintf(buf, sizeof(buf),
               "f64 nmax<=%d lmax=%d coef tiles %dx%d (groups %d|%d, tiles/lane %d|%d); block "
               "variant %d x %d tiles, %d groups, %d particles per stage",
               NMAXC, LMAX, S0::NR, S0::JT, S0::G, S2::G, S0::KT, S2::KT, BS::NR, BS::JT, BS::G,
               BS::P);
    }
    return buf;
  }
};

}  // namespace scf
