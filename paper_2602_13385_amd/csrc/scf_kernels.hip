// HIP kernels of the SCF hot path for gfx950 (MI355X).
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
#include <hip/hip_runtime.h>

#include <cstdio>

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
  static constexpr int ACC_MAX = sizeof(R) == 4 ? 96 : 64;
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
  R bl[KT][NR];
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

  R acc[KT][NR][JT];
#pragma unroll
  for (int k = 0; k < KT; ++k)
#pragma unroll
    for (int i = 0; i < NR; ++i)
#pragma unroll
      for (int j = 0; j < JT; ++j) acc[k][i][j] = R(0);

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
    if (q < P && gi < end) {
      nx = a.x[gi];
      ny = a.y[gi];
      nz = a.z[gi];
      nm = a.m[gi];
    }
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
        const R m2 = R(mc) * R(mc);
        R Q0 = R(0), Q1 = R(0);
#pragma unroll
        for (int l = kk * LPP; l <= LMAX; ++l) {
          // gamma_lm = ((l-1)^2 - m^2) / ((2l-1)(2l-3)), used for l >= m+2
          const R cl = l >= 2 ? R(1) / R((2 * l - 1) * (2 * l - 3)) : R(0);
          const R gam = fma(-m2, cl, R((l - 1) * (l - 1)) * cl);
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
        nx = a.x[gi];
        ny = a.y[gi];
        nz = a.z[gi];
        nm = a.m[gi];
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
    for (int gg = 1; gg < G; ++gg) {
      if (grp == gg && tv[0]) {
        R* dst = rec + tt[0] * NR * JT;
#pragma unroll
        for (int i = 0; i < NR; ++i)
#pragma unroll
          for (int j = 0; j < JT; ++j) dst[i * JT + j] = acc[0][i][j];
      }
      stage_sync<WPB>();
      if (grp == 0 && tv[0]) {
        const R* src = rec + tt[0] * NR * JT;
#pragma unroll
        for (int i = 0; i < NR; ++i)
#pragma unroll
          for (int j = 0; j < JT; ++j) acc[0][i][j] += src[i * JT + j];
      }
      stage_sync<WPB>();
    }
  }
  R* out = a.partials + ((int64_t)slot * ROWS + (LDS_COMBINE ? 0 : grp)) * a.T;
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

template <typename R, int NMAXC, int LMAX, int MODE, bool BATCHED>
__global__ void __launch_bounds__(256) field_kernel(ForceArgs<R> a) {
  constexpr int L1 = LMAX + 1, NW = NMAXC + 1;
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
  const R* __restrict__ bR = a.beta_rad;
  const R* __restrict__ bA = a.beta_ang;
  const R x = a.x[i], y = a.y[i], z = a.z[i];
  Geom<R> g = make_geom<R>(x, y, z, a.binv, a.alpha, a.inv_alpha, a.amode);

  R Er[L1], Ei[L1];
  Er[0] = R(1);
  Ei[0] = R(0);
#pragma unroll
  for (int m = 1; m <= LMAX; ++m) {
    Er[m] = Er[m - 1] * g.ux - Ei[m - 1] * g.uy;
    Ei[m] = Er[m - 1] * g.uy + Ei[m - 1] * g.ux;
  }
  R Qm1[L1], Qm2[L1], dQm1[L1], dQm2[L1];
#pragma unroll
  for (int m = 0; m <= LMAX; ++m) Qm1[m] = Qm2[m] = dQm1[m] = dQm2[m] = R(0);
  R psi = R(0), psir = R(0), gx = R(0), gy = R(0), gz = R(0);
  R Gprev = R(0), Gl = g.g0;
  // The degree loop is a real (wave-uniform) loop so that only one degree's
  // radial vector is live; the order loop is unrolled with uniform exits.
#pragma unroll 1
  for (int l = 0; l <= LMAX; ++l) {
    if (l > 0) {
      Gprev = Gl;
      Gl = Gl * g.w;
    }
    const R fl = R(l);
    const R dGl = fl * Gprev * g.om - (R(2) * fl + R(1)) * g.kap * Gl;
    // radial basis p_n and dp_n/dxi
    R p[NW], dp[NW];
    p[0] = R(1);
    dp[0] = R(0);
    if constexpr (NMAXC >= 1) {
      p[1] = g.xi;
      dp[1] = R(1);
    }
    const R* __restrict__ bRl = bR + l * NW;
#pragma unroll
    for (int n = 2; n <= NMAXC; ++n) {
      const R b = bRl[n];
      p[n] = g.xi * p[n - 1] - b * p[n - 2];
      dp[n] = fma(g.xi, dp[n - 1], p[n - 1]) - b * dp[n - 2];
    }
    R psl = R(0), rhl = R(0), gxl = R(0), gyl = R(0), gzl = R(0);
    const R* __restrict__ Wl = W + l * l * NW;
#pragma unroll
    for (int m = 0; m <= LMAX; ++m) {
      if (m > l) break;
      R Q, dQ;
      if (l == m) {
        Q = R(1);
        dQ = R(0);
      } else if (l == m + 1) {
        Q = g.c;
        dQ = R(1);
      } else {
        const R b = bA[m * L1 + l];
        Q = g.c * Qm1[m] - b * Qm2[m];
        dQ = fma(g.c, dQm1[m], Qm1[m]) - b * dQm2[m];
      }
      Qm2[m] = Qm1[m];
      Qm1[m] = Q;
      dQm2[m] = dQm1[m];
      dQm1[m] = dQ;
      const R* __restrict__ wc = Wl + (m == 0 ? 0 : 2 * m - 1) * NW;
      R sc = wc[0], dsc = R(0);
      if constexpr (NMAXC >= 1) {
        sc = fma(wc[1], p[1], sc);
        dsc = wc[1];
      }
#pragma unroll
      for (int n = 2; n <= NMAXC; ++n) {
        sc = fma(wc[n], p[n], sc);
        dsc = fma(wc[n], dp[n], dsc);
      }
      if (m == 0) {
        psl = fma(Q, sc, psl);
        rhl = fma(Q, dsc, rhl);
        gzl = fma(dQ, sc, gzl);
      } else {
        const R* __restrict__ ws = wc + NW;
        R ss = ws[0], dss = R(0);
        if constexpr (NMAXC >= 1) {
          ss = fma(ws[1], p[1], ss);
          dss = ws[1];
        }
#pragma unroll
        for (int n = 2; n <= NMAXC; ++n) {
          ss = fma(ws[n], p[n], ss);
          dss = fma(ws[n], dp[n], dss);
        }
        const R v1 = sc * Er[m] + ss * Ei[m];
        const R v2 = dsc * Er[m] + dss * Ei[m];
        const R v3 = sc * Er[m - 1] + ss * Ei[m - 1];
        const R v4 = ss * Er[m - 1] - sc * Ei[m - 1];
        const R mQ = R(m) * Q;
        psl = fma(Q, v1, psl);
        rhl = fma(Q, v2, rhl);
        gzl = fma(dQ, v1, gzl);
        gxl = fma(mQ, v3, gxl);
        gyl = fma(mQ, v4, gyl);
      }
    }
    psi = fma(Gl, psl, psi);
    psir = fma(dGl, psl, fma(Gl * g.dxi, rhl, psir));
    gx = fma(Gl, gxl, gx);
    gy = fma(Gl, gyl, gy);
    gz = fma(Gl, gzl, gz);
  }
  // grad psi = psi_r rhat + (1/r) (Gamma - (rhat . Gamma) rhat)
  const R rg = g.ux * gx + g.uy * gy + g.c * gz;
  R axv = R(0), ayv = R(0), azv = R(0);
  if (g.r > R(0)) {
    axv = -(psir * g.ux + g.ir * (gx - rg * g.ux));
    ayv = -(psir * g.uy + g.ir * (gy - rg * g.uy));
    azv = -(psir * g.c + g.ir * (gz - rg * g.c));
  }
  if (a.host.ncomp > 0) {
    R hx, hy, hz;
    host_grad<R>(a.host, cx + x, cy + y, cz + z, hx, hy, hz);
    axv += gcx - hx;
    ayv += gcy - hy;
    azv += gcz - hz;
  }
  if (MODE == 0) {
    a.ax[i] = axv;
    a.ay[i] = ayv;
    a.az[i] = azv;
    if (a.pot) a.pot[i] = psi;
  } else {
    R vx = fma(a.kick, axv, a.vx[i]);
    R vy = fma(a.kick, ayv, a.vy[i]);
    R vz = fma(a.kick, azv, a.vz[i]);
    a.vx[i] = vx;
    a.vy[i] = vy;
    a.vz[i] = vz;
    a.ax[i] = axv;
    a.ay[i] = ayv;
    a.az[i] = azv;
    if (a.drift != R(0)) {
      a.x[i] = fma(a.drift, vx, x);
      a.y[i] = fma(a.drift, vy, y);
      a.z[i] = fma(a.drift, vz, z);
    }
  }
}

// ---------------------------------------------------------------------------
// small kernels
// ---------------------------------------------------------------------------
// partial sums over blocks: red1[chunk][t] = sum_{b in chunk} partials[b][t] (double)
template <typename R>
__global__ void __launch_bounds__(256) reduce_kernel(const R* __restrict__ partials, int nblocks,
                                                     int T, int per_chunk, double* red1) {
  __shared__ double sh[4][64];
  const int ti = threadIdx.x & 63, kc = threadIdx.x >> 6;
  const int t = blockIdx.x * 64 + ti;
  const int b0 = blockIdx.y * per_chunk;
  int b1 = b0 + per_chunk;
  if (b1 > nblocks) b1 = nblocks;
  double s = 0.0;
  if (t < T)
    for (int b = b0 + kc; b < b1; b += 4) s += double(partials[(int64_t)b * T + t]);
  sh[kc][ti] = s;
  __syncthreads();
  if (kc == 0 && t < T)
    red1[(int64_t)blockIdx.y * T + t] = ((sh[0][ti] + sh[1][ti]) + sh[2][ti]) + sh[3][ti];
}

template <typename R>
__global__ void __launch_bounds__(256) finalize_kernel(const double* __restrict__ red1, int nchunks,
                                                       int T, int nmax, int lmax, int nmaxc,
                                                       const double* __restrict__ cs,
                                                       const double* __restrict__ fw, double* coef,
                                                       R* W) {
  const int L2 = (lmax + 1) * (lmax + 1);
  const int e = blockIdx.x * blockDim.x + threadIdx.x;  // over (NMAXC+1) * L2 W entries
  if (e >= (nmaxc + 1) * L2) return;
  const int lj = e / (nmaxc + 1), n = e % (nmaxc + 1);
  if (n > nmax) {
    W[e] = R(0);
    return;
  }
  const int t = n * L2 + lj;
  double s = 0.0;
  for (int c = 0; c < nchunks; ++c) s += red1[(int64_t)c * T + t];
  const double cv = cs[t] * s;
  if (coef) coef[t] = cv;
  W[e] = R(fw[t] * cv);
}

template <typename R>
__global__ void __launch_bounds__(256) make_w_kernel(const double* __restrict__ coef, int T, int nmax,
                                                     int lmax, int nmaxc,
                                                     const double* __restrict__ fw, R* W) {
  const int L2 = (lmax + 1) * (lmax + 1);
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (nmaxc + 1) * L2) return;
  const int lj = e / (nmaxc + 1), n = e % (nmaxc + 1);
  if (n > nmax) {
    W[e] = R(0);
    return;
  }
  const int t = n * L2 + lj;
  W[e] = R(fw[t] * coef[t]);
}

template <typename R>
__global__ void __launch_bounds__(256) kick_drift_kernel(int64_t n, R* x, R* y, R* z, R* vx, R* vy,
                                                         R* vz, const R* ax, const R* ay,
                                                         const R* az, R kick, R drift) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  R u = fma(kick, ax[i], vx[i]), v = fma(kick, ay[i], vy[i]), w = fma(kick, az[i], vz[i]);
  vx[i] = u;
  vy[i] = v;
  vz[i] = w;
  x[i] = fma(drift, u, x[i]);
  y[i] = fma(drift, v, y[i]);
  z[i] = fma(drift, w, z[i]);
}

// Batched reduction: cluster c owns partial rows [rows[c], rows[c+1]);
// red1[c][chunk][t] sums its rows of one chunk (double).
template <typename R>
__global__ void __launch_bounds__(256) reduce_batched_kernel(const R* __restrict__ partials,
                                                             const int32_t* __restrict__ rows,
                                                             int T, int nchunks, double* red1) {
  __shared__ double sh[4][64];
  const int ti = threadIdx.x & 63, kc = threadIdx.x >> 6;
  const int t = blockIdx.x * 64 + ti;
  const int c = blockIdx.z;
  const int r0 = rows[c], r1 = rows[c + 1];
  const int per_chunk = (r1 - r0 + nchunks - 1) / nchunks;
  const int b0 = r0 + blockIdx.y * per_chunk;
  int b1 = b0 + per_chunk;
  if (b1 > r1) b1 = r1;
  double s = 0.0;
  if (t < T)
    for (int b = b0 + kc; b < b1; b += 4) s += double(partials[(int64_t)b * T + t]);
  sh[kc][ti] = s;
  __syncthreads();
  if (kc == 0 && t < T)
    red1[((int64_t)c * nchunks + blockIdx.y) * T + t] =
        ((sh[0][ti] + sh[1][ti]) + sh[2][ti]) + sh[3][ti];
}

// Batched finalisation: coef[c][t] and W[c][.] of every cluster.  Block
// (0, 0) also copies row *step of the centre table into cur (the rows the
// field pass of this step reads) and then advances *step.
template <typename R>
__global__ void __launch_bounds__(256) finalize_batched_kernel(
    const double* __restrict__ red1, int nchunks, int T, int nmax, int lmax, int nmaxc,
    const double* __restrict__ cs, const double* __restrict__ fw, double* coef, R* W,
    int64_t W_stride, const double* __restrict__ centre_tab, int ncl, double* cur, int* step) {
  const int L2 = (lmax + 1) * (lmax + 1);
  const int c = blockIdx.y;
  if (blockIdx.x == 0 && c == 0 && step) {
    const int k = *step;
    for (int i = threadIdx.x; i < ncl * 9; i += blockDim.x)
      cur[i] = centre_tab[(int64_t)k * ncl * 9 + i];
    __syncthreads();
    if (threadIdx.x == 0) *step = k + 1;
  }
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (nmaxc + 1) * L2) return;
  R* Wc = W + (int64_t)c * W_stride;
  const int lj = e / (nmaxc + 1), n = e % (nmaxc + 1);
  if (n > nmax) {
    Wc[e] = R(0);
    return;
  }
  const int t = n * L2 + lj;
  const double* r = red1 + (int64_t)c * nchunks * T;
  double s = 0.0;
  for (int ch = 0; ch < nchunks; ++ch) s += r[(int64_t)ch * T + t];
  const double cv = cs[t] * s;
  if (coef) coef[(int64_t)c * T + t] = cv;
  Wc[e] = R(fw[t] * cv);
}

__global__ void set_int_kernel(int* p, int v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

__global__ void fill_kernel(double* p, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_reduce(int dtype, const void* partials, int nblocks, int T, int nchunks,
                         double* red1, hipStream_t s) {
  if (nblocks <= 0 || T <= 0) return hipSuccess;
  const int per_chunk = (nblocks + nchunks - 1) / nchunks;
  dim3 grid((T + 63) / 64, nchunks);
  if (dtype == 0)
    reduce_kernel<float><<<grid, 256, 0, s>>>((const float*)partials, nblocks, T, per_chunk, red1);
  else
    reduce_kernel<double><<<grid, 256, 0, s>>>((const double*)partials, nblocks, T, per_chunk, red1);
  return hipGetLastError();
}

hipError_t launch_finalize(int dtype, const double* red1, int nchunks, int T, int nmax, int lmax,
                           int nmaxc, const double* cs, const double* fw, double* coef, void* W,
                           hipStream_t s) {
  const int ne = (nmaxc + 1) * (lmax + 1) * (lmax + 1);
  const int grid = (ne + 255) / 256;
  if (dtype == 0)
    finalize_kernel<float><<<grid, 256, 0, s>>>(red1, nchunks, T, nmax, lmax, nmaxc, cs, fw, coef,
                                                (float*)W);
  else
    finalize_kernel<double><<<grid, 256, 0, s>>>(red1, nchunks, T, nmax, lmax, nmaxc, cs, fw, coef,
                                                 (double*)W);
  return hipGetLastError();
}

hipError_t launch_make_w(int dtype, const double* coef, int T, int nmax, int lmax, int nmaxc,
                         const double* fw, void* W, hipStream_t s) {
  const int ne = (nmaxc + 1) * (lmax + 1) * (lmax + 1);
  const int grid = (ne + 255) / 256;
  if (dtype == 0)
    make_w_kernel<float><<<grid, 256, 0, s>>>(coef, T, nmax, lmax, nmaxc, fw, (float*)W);
  else
    make_w_kernel<double><<<grid, 256, 0, s>>>(coef, T, nmax, lmax, nmaxc, fw, (double*)W);
  return hipGetLastError();
}

hipError_t launch_kick_drift(int dtype, int64_t n, void* x, void* y, void* z, void* vx, void* vy,
                             void* vz, const void* ax, const void* ay, const void* az, double kick,
                             double drift, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t grid = (n + 255) / 256;
  if (dtype == 0)
    kick_drift_kernel<float><<<dim3((unsigned)grid), 256, 0, s>>>(
        n, (float*)x, (float*)y, (float*)z, (float*)vx, (float*)vy, (float*)vz, (const float*)ax,
        (const float*)ay, (const float*)az, (float)kick, (float)drift);
  else
    kick_drift_kernel<double><<<dim3((unsigned)grid), 256, 0, s>>>(
        n, (double*)x, (double*)y, (double*)z, (double*)vx, (double*)vy, (double*)vz,
        (const double*)ax, (const double*)ay, (const double*)az, kick, drift);
  return hipGetLastError();
}

hipError_t launch_reduce_batched(int dtype, const void* partials, const int32_t* rows, int ncl,
                                 int T, int nchunks, double* red1, hipStream_t s) {
  if (ncl <= 0 || T <= 0) return hipSuccess;
  dim3 grid((T + 63) / 64, nchunks, ncl);
  if (dtype == 0)
    reduce_batched_kernel<float><<<grid, 256, 0, s>>>((const float*)partials, rows, T, nchunks, red1);
  else
    reduce_batched_kernel<double><<<grid, 256, 0, s>>>((const double*)partials, rows, T, nchunks,
                                                       red1);
  return hipGetLastError();
}

hipError_t launch_finalize_batched(int dtype, const double* red1, int nchunks, int T, int nmax,
                                   int lmax, int nmaxc, const double* cs, const double* fw,
                                   double* coef, void* W, int64_t W_stride,
                                   const double* centre_tab, int ncl, double* cur, int* step,
                                   hipStream_t s) {
  if (ncl <= 0) return hipSuccess;
  const int ne = (nmaxc + 1) * (lmax + 1) * (lmax + 1);
  dim3 grid((ne + 255) / 256, ncl);
  if (dtype == 0)
    finalize_batched_kernel<float><<<grid, 256, 0, s>>>(red1, nchunks, T, nmax, lmax, nmaxc, cs, fw,
                                                        coef, (float*)W, W_stride, centre_tab, ncl,
                                                        cur, step);
  else
    finalize_batched_kernel<double><<<grid, 256, 0, s>>>(red1, nchunks, T, nmax, lmax, nmaxc, cs,
                                                         fw, coef, (double*)W, W_stride,
                                                         centre_tab, ncl, cur, step);
  return hipGetLastError();
}

hipError_t launch_set_int(int* p, int v, hipStream_t s) {
  set_int_kernel<<<1, 64, 0, s>>>(p, v);
  return hipGetLastError();
}

hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  fill_kernel<<<dim3((unsigned)((n + 255) / 256)), 256, 0, s>>>(p, n, v);
  return hipGetLastError();
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

template <typename R, int NMAXC, int LMAX>
struct EngineImpl final : Engine {
  using V = CoefVariants<R>;
  int nmaxc() const override { return NMAXC; }
  int lmax() const override { return LMAX; }
  int dtype() const override { return sizeof(R) == 4 ? 0 : 1; }
  size_t real_size() const override { return sizeof(R); }
  int coef_variants() const override { return V::N; }
  int stage_particles(int v) const override { return 64 / V::LPP[v]; }
  int rows_per_unit(int v) const override {
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
  int waves_per_block(int v) const override { return V::WPB[v]; }
  hipError_t launch_coef(const void* args, int nunits, int v, hipStream_t s) const override {
    if (nunits <= 0) return hipSuccess;
    const CoefArgs<R>& ca = *(const CoefArgs<R>*)args;
    const int wpb = V::WPB[v];
    const int nblocks = (nunits + wpb - 1) / wpb;
    if (v == 0)
      coef_kernel<R, NMAXC, LMAX, V::LPP[0], V::WPB[0]><<<nblocks, 64 * V::WPB[0], 0, s>>>(ca);
    else if (v == 1)
      coef_kernel<R, NMAXC, LMAX, V::LPP[1], V::WPB[1]><<<nblocks, 64 * V::WPB[1], 0, s>>>(ca);
    else
      coef_kernel<R, NMAXC, LMAX, V::LPP[2], V::WPB[2]><<<nblocks, 64 * V::WPB[2], 0, s>>>(ca);
    return hipGetLastError();
  }
  hipError_t launch_force(const void* args, int64_t nblocks, int mode,
                          hipStream_t s) const override {
    if (nblocks <= 0) return hipSuccess;
    const ForceArgs<R>& fa = *(const ForceArgs<R>*)args;
    if (fa.blk_cluster)
      field_kernel<R, NMAXC, LMAX, 1, true><<<dim3((unsigned)nblocks), 256, 0, s>>>(fa);
    else if (mode == 0)
      field_kernel<R, NMAXC, LMAX, 0, false><<<dim3((unsigned)nblocks), 256, 0, s>>>(fa);
    else
      field_kernel<R, NMAXC, LMAX, 1, false><<<dim3((unsigned)nblocks), 256, 0, s>>>(fa);
    return hipGetLastError();
  }
  const char* describe() const override {
    static char buf[200];
    using S0 = CoefShape<R, NMAXC, LMAX, V::LPP[0]>;
    using S2 = CoefShape<R, NMAXC, LMAX, V::LPP[2]>;
    snprintf(buf, sizeof(buf),
             "%s nmax<=%d lmax=%d coef tiles %dx%d (groups %d|%d, tiles/lane %d|%d)",
             sizeof(R) == 4 ? "f32" : "f64", NMAXC, LMAX, S0::NR, S0::JT, S0::G, S2::G, S0::KT,
             S2::KT);
    return buf;
  }
};

#define SCF_ENGINE(R, N, L)                      \
  if (nmax <= N && lmax == L && exact == (N == nmax)) { \
    static EngineImpl<R, N, L> e;                \
    return &e;                                   \
  }

template <typename R>
static Engine* find_engine_t(int nmax, int lmax, bool exact) {
  // exact-size instances for the shipped workloads
  SCF_ENGINE(R, 6, 4)
  SCF_ENGINE(R, 10, 5)
  SCF_ENGINE(R, 10, 6)
  SCF_ENGINE(R, 16, 10)
  // generic instances: any nmax <= 20 for these degrees
  SCF_ENGINE(R, 20, 0)
  SCF_ENGINE(R, 20, 1)
  SCF_ENGINE(R, 20, 2)
  SCF_ENGINE(R, 20, 3)
  SCF_ENGINE(R, 20, 4)
  SCF_ENGINE(R, 20, 5)
  SCF_ENGINE(R, 20, 6)
  SCF_ENGINE(R, 20, 8)
  SCF_ENGINE(R, 20, 10)
  return nullptr;
}
#undef SCF_ENGINE

Engine* find_engine(int dtype, int nmax, int lmax) {
  if (nmax < 0 || lmax < 0) return nullptr;
  Engine* e = dtype == 0 ? find_engine_t<float>(nmax, lmax, true) : find_engine_t<double>(nmax, lmax, true);
  if (e) return e;
  return dtype == 0 ? find_engine_t<float>(nmax, lmax, false) : find_engine_t<double>(nmax, lmax, false);
}

}  // namespace scf
