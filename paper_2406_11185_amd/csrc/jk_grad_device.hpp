// Nuclear-gradient kernel of the J/K energy E = 1/2 tr(DJ) - 1/4 tr(DK) at
// fixed D, for gfx950.  Shares the pair data, Boys tables, screening and work
// items of the J/K build; the per-class code comes from gen_grad.py.
#pragma once
#include "jk_classes.hpp"

namespace jk {

struct GradLaunch {
  EriLaunch e;      // pair data, items, D, Boys tables (J, K unused)
  double* dEdR;     // [n_dm][n_atoms][3]
  int n_atoms;
  void* ws;         // workspace: nwaves * 64 lanes * C::WS values of type T
  int nwaves;       // wavefronts of the launch; each claims items until none is left
  int lds_doubles;  // n_dm * n_atoms * 3 when the workgroup accumulates dE/dR in LDS,
                    // else 0; dynamic shared memory of lds_bytes (8 bytes per value, or
                    // two int64 words per value in deterministic mode)
  size_t lds_bytes;
};

// Gradient contributions go to a workgroup copy of dE/dR in LDS (the whole
// gradient is a few hundred values, so direct global atomics from every
// quartet would serialise on a handful of lines) and are added to global
// memory once per workgroup at the end; without LDS room, directly.
// Deterministic mode (det_lo > 0): dEdR points to int64 fixed-point pairs (see
// atomic_add) and the LDS copy holds the same pairs, lo words nl values after
// the hi words.
__device__ __forceinline__ void grad_add(double* lds, double* glob, int idx, double v,
                                         size_t det_lo, int nl) {
  if (!lds) {
    atomic_add(&glob[idx], v, det_lo);
  } else if (det_lo == 0) {
    atomicAdd(&lds[idx], v);
  } else {
    const double s = v * kFixHi;
    const double h = rint(s);
    unsigned long long* w = reinterpret_cast<unsigned long long*>(lds);
    atomicAdd(&w[idx], static_cast<unsigned long long>(static_cast<long long>(h)));
    atomicAdd(&w[idx + nl],
              static_cast<unsigned long long>(static_cast<long long>(rint((s - h) * kFixLo))));
  }
}



// Contraction loop with the exponent weights of the derivative integrals:
// wA = 2a, wB = 2b (bra primitives), wC = 2c (first ket primitive).
// The G lanes of a group split the primitive quartets (sub, sub+G, ...).
template <int L, typename T, int G, class V>
__device__ __forceinline__ void contract_w(const EriLaunch& a, int i, int k, int sub, T ACx,
                                           T ACy, T ACz, V&& vrr) {
  const int nb = a.bra.n, nk = a.ket.n;
  const int nppb = a.bra.npp, nppk = a.ket.npp;
  const int npq = nppb * nppk;
  for (int pq = sub; pq < npq; pq += G) {
    const int kl = pq / nppb, ij = pq - kl * nppb;
    const T* kp = prim_of<T>(a.ket) + static_cast<size_t>(kl) * kPrimFields * nk + k;
    const T* bp = prim_of<T>(a.bra) + static_cast<size_t>(ij) * kPrimFields * nb + i;
    T F[L + 1];
    VrrCoef<T> c;
    prim_setup<L, T>(T(bp[kP * nb]), T(bp[kOo2p * nb]), T(bp[kPAx * nb]), T(bp[kPAy * nb]),
                     T(bp[kPAz * nb]), T(bp[kKt * nb]), T(kp[kP * nk]), T(kp[kOo2p * nk]),
                     T(kp[kPAx * nk]), T(kp[kPAy * nk]), T(kp[kPAz * nk]), T(kp[kKt * nk]), ACx,
                     ACy, ACz, a, F, c);
    vrr(F, c, T(bp[kTwoA * nb]), T(bp[kTwoB * nb]), T(kp[kTwoA * nk]));
  }
}

template <class C, typename T, int GL, int J>
__device__ __forceinline__ void grad_pass_body(const EriLaunch& a, int i, int k, int sub, T ACx,
                                               T ACy, T ACz, LaneArr<T, kWave / GL> G, int z) {
  constexpr int N = C::template Pass<J>::N;
  T acc[N];
#pragma unroll
  for (int t = 0; t < N; ++t) acc[t] = T(0);
  contract_w<C::L, T, GL>(a, i, k, sub, ACx, ACy, ACz,
                          [&](const T* F, const VrrCoef<T>& c, T wA, T wB, T wC) {
                            C::template vrr_pass<J, T>(F, c, wA, wB, wC, acc);
                          });
  group_sum_all<GL>(acc);
  if (sub == 0) C::template store_pass<J, T, LaneArr<T, kWave / GL>>(acc, G, z);
}

// Classes with many passes call each pass as a separate function, so that the
// compiler allocates registers pass by pass.
template <class C, typename T, int GL, int J>
__device__ __attribute__((noinline)) void grad_pass_call(const EriLaunch& a, int i, int k, int sub,
                                                          T ACx, T ACy, T ACz,
                                                          LaneArr<T, kWave / GL> G, int z) {
  grad_pass_body<C, T, GL, J>(a, i, k, sub, ACx, ACy, ACz, G, z);
}

template <class C, typename T, int GL, int J>
__device__ __forceinline__ void grad_passes(const EriLaunch& a, int i, int k, int sub, T ACx,
                                            T ACy, T ACz, LaneArr<T, kWave / GL> G, int z) {
  if constexpr (C::NPASS > 4)
    grad_pass_call<C, T, GL, J>(a, i, k, sub, ACx, ACy, ACz, G, z);
  else
    grad_pass_body<C, T, GL, J>(a, i, k, sub, ACx, ACy, ACz, G, z);
  if constexpr (J + 1 < C::NPASS) grad_passes<C, T, GL, J + 1>(a, i, k, sub, ACx, ACy, ACz, G, z);
}

constexpr int at_least_1(int v) { return v > 0 ? v : 1; }

// One wavefront per work item; bra pair uniform, one ket pair per lane.
template <class C, typename T, int GL>
__global__ __launch_bounds__(kBlock) void grad_kernel(const GradLaunch g) {
  constexpr int NCD = C::NC * C::ND;
  constexpr int NAB = C::NA * C::NB;
  const EriLaunch& a = g.e;
  constexpr int QPW = kWave / GL;
  const int lane = threadIdx.x & (kWave - 1);
  const int sub = lane & (GL - 1), ql = lane / GL;
  const int wave = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  extern __shared__ double gacc[];   // [n_dm][n_atoms][3] when g.lds_doubles > 0
  double* const lds = g.lds_doubles > 0 ? gacc : nullptr;
  const size_t det = a.det_lo;
  const int nl = g.lds_doubles;
  if (lds) {
    for (int t = threadIdx.x; t < (det ? 2 : 1) * nl; t += kBlock) gacc[t] = 0.0;
    __syncthreads();
  }
  // waves past the launch's wavefront count only take part in the final flush
  const bool idle = wave >= g.nwaves;
  using AT = LaneArr<T, QPW>;
  T* wsl = static_cast<T*>(g.ws) + static_cast<size_t>(idle ? 0 : wave) * C::WS * QPW + ql;
  const AT G{wsl};
  const AT XA{wsl + static_cast<size_t>(C::NG) * QPW};
  const AT XB{XA.p + static_cast<size_t>(C::NE_A) * NCD * QPW};
  const AT XC{XB.p + static_cast<size_t>(C::NE_B) * NCD * QPW};
  const AT XU{XC.p + static_cast<size_t>(C::NE_C) * C::NCP * QPW};
  const AT XV{XU.p + static_cast<size_t>(C::NE_U) * NCD * QPW};
  const int z = 0;
  for (int item = idle ? a.nitems : claim_item(a.next); item < a.nitems; item = claim_item(a.next)) {
  const int4 w = a.items[item];
  const int i = __builtin_amdgcn_readfirstlane(w.x);
  const int kbeg = __builtin_amdgcn_readfirstlane(w.y);
  const int kend = __builtin_amdgcn_readfirstlane(w.z);
  const int nb = a.bra.n, nk = a.ket.n;
  const size_t n = static_cast<size_t>(a.n);
  const size_t nn = n * n;
  const double Ax = a.bra.A[i], Ay = a.bra.A[nb + i], Az = a.bra.A[2 * nb + i];
  const T ABx = T(a.bra.AB[i]), ABy = T(a.bra.AB[nb + i]), ABz = T(a.bra.AB[2 * nb + i]);
  const int a0 = a.bra.bf[i], b0 = a.bra.bf[nb + i];
  const int atA = a.bra.atoms[i], atB = a.bra.atoms[nb + i];
  const double fbra = a.bra.fpair[i];

  for (int kc = kbeg; kc < kend; kc += QPW) {
    const bool inrange = kc + ql < kend;
    const bool active = inrange && sub == 0;
    const int k = inrange ? kc + ql : kend - 1;
    const T ACx = T(Ax - a.ket.A[k]), ACy = T(Ay - a.ket.A[nk + k]),
            ACz = T(Az - a.ket.A[2 * nk + k]);
    grad_passes<C, T, GL, 0>(a, i, k, sub, ACx, ACy, ACz, G, z);
    const T CDx = T(a.ket.AB[k]), CDy = T(a.ket.AB[nk + k]), CDz = T(a.ket.AB[2 * nk + k]);

    // ket horizontal recurrences, one bra index e at a time; the G lanes of a
    // quartet share them (e = sub, sub+G, ...) and then the (c, d) loop
    lanes_sync();   // the passes were stored by the group's first lane
#pragma nounroll
    for (int e = sub; e < C::NE_A; e += GL) {
      T f[C::NF_A], o[NCD];
#pragma unroll
      for (int t = 0; t < C::NF_A; ++t) f[t] = G[z + C::OFF_A + e * C::NF_A + t];
      C::template ket_b<T>(f, CDx, CDy, CDz, o);
#pragma unroll
      for (int t = 0; t < NCD; ++t) XA[z + e * NCD + t] = o[t];
    }
#pragma nounroll
    for (int e = sub; e < C::NE_B; e += GL) {
      T f[C::NF_B], o[NCD];
#pragma unroll
      for (int t = 0; t < C::NF_B; ++t) f[t] = G[z + C::OFF_B + e * C::NF_B + t];
      C::template ket_b<T>(f, CDx, CDy, CDz, o);
#pragma unroll
      for (int t = 0; t < NCD; ++t) XB[z + e * NCD + t] = o[t];
    }
#pragma nounroll
    for (int e = sub; e < C::NE_C; e += GL) {
      T f[C::NF_C], o[C::NCP];
#pragma unroll
      for (int t = 0; t < C::NF_C; ++t) f[t] = G[z + C::OFF_C + e * C::NF_C + t];
      C::template ket_p<T>(f, CDx, CDy, CDz, o);
#pragma unroll
      for (int t = 0; t < C::NCP; ++t) XC[z + e * C::NCP + t] = o[t];
    }
    if constexpr (C::USE_U) {
#pragma nounroll
      for (int e = sub; e < C::NE_U; e += GL) {
        T f[C::NF_U], o[NCD];
#pragma unroll
        for (int t = 0; t < C::NF_U; ++t) f[t] = G[z + C::OFF_U + e * C::NF_U + t];
        C::template ket_b<T>(f + C::U_FB, CDx, CDy, CDz, o);
#pragma unroll
        for (int t = 0; t < NCD; ++t) XU[z + e * NCD + t] = o[t];
        if constexpr (C::NCM > 0) {
          T om[at_least_1(C::NCM)];
          C::template ket_m<T>(f, CDx, CDy, CDz, om);
#pragma unroll
          for (int t = 0; t < C::NCM; ++t) XV[z + e * C::NCM + t] = om[t];
        }
      }
    }

    lanes_sync();   // the transformed rows come from all lanes of the group
    const int c0 = a.ket.bf[k], d0 = a.ket.bf[nk + k];
    const int atC = a.ket.atoms[k], atD = a.ket.atoms[nk + k];
    const double fq =
        inrange ? 8.0 * fbra * a.ket.fpair[k] * ((a.same_bin && k == i) ? 0.5 : 1.0) : 0.0;

    for (int m = 0; m < a.n_dm; ++m) {
      const double* Dm = a.D + m * nn;
      double Dab[NAB];
#pragma unroll
      for (int x = 0; x < C::NA; ++x)
#pragma unroll
        for (int y = 0; y < C::NB; ++y) Dab[x * C::NB + y] = Dm[(a0 + x) * n + b0 + y];
      double gA[3] = {0.0, 0.0, 0.0}, gB[3] = {0.0, 0.0, 0.0}, gC[3] = {0.0, 0.0, 0.0};
#pragma nounroll
      for (int cd = sub; cd < NCD; cd += GL) {
        const int c = cd / C::ND, d = cd % C::ND;
        const double Dcd = Dm[(c0 + c) * n + d0 + d];
        double Dac[C::NA], Dad[C::NA], Dbc[C::NB], Dbd[C::NB];
#pragma unroll
        for (int x = 0; x < C::NA; ++x) {
          Dac[x] = Dm[(a0 + x) * n + c0 + c];
          Dad[x] = Dm[(a0 + x) * n + d0 + d];
        }
#pragma unroll
        for (int y = 0; y < C::NB; ++y) {
          Dbc[y] = Dm[(b0 + y) * n + c0 + c];
          Dbd[y] = Dm[(b0 + y) * n + d0 + d];
        }
        double Gam[NAB];
#pragma unroll
        for (int x = 0; x < C::NA; ++x)
#pragma unroll
          for (int y = 0; y < C::NB; ++y)
            Gam[x * C::NB + y] = 0.5 * Dab[x * C::NB + y] * Dcd -
                                 0.125 * (Dac[x] * Dbd[y] + Dad[x] * Dbc[y]);
        // centres A and B
        T ea[C::NE_A], eb[C::NE_B];
#pragma unroll
        for (int e = 0; e < C::NE_A; ++e) ea[e] = XA[z + e * NCD + cd];
#pragma unroll
        for (int e = 0; e < C::NE_B; ++e) eb[e] = XB[z + e * NCD + cd];
        T xap[(C::NA + C::LA + 2) * C::NB + 8], xbp[C::NA * (C::NB + C::LB + 2) + 8];
        C::template bra_ap<T>(ea, ABx, ABy, ABz, xap);
        C::template bra_bp<T>(eb, ABx, ABy, ABz, xbp);
        T xam[at_least_1(C::LA >= 1 ? C::NA * C::NB : 0)];
        T xbm[at_least_1(C::LB >= 1 ? C::NA * C::NB : 0)];
        if constexpr (C::LA >= 1) {
          T em[at_least_1(C::NE_AM)];
#pragma unroll
          for (int e = 0; e < C::NE_AM; ++e) em[e] = XU[z + e * NCD + cd];
          C::template bra_am<T>(em, ABx, ABy, ABz, xam);
        }
        if constexpr (C::LB >= 1) {
          T em[at_least_1(C::NE_BM)];
#pragma unroll
          for (int e = 0; e < C::NE_BM; ++e) em[e] = XU[z + (C::U_EB + e) * NCD + cd];
          C::template bra_bm<T>(em, ABx, ABy, ABz, xbm);
        }
        C::template contract_ab<T>(Gam, xap, xam, xbp, xbm, gA, gB);
        // centre C
#pragma unroll
        for (int x = 0; x < 3; ++x) {
          const int cp = C::CPLUS[c][x];
          T e0[C::NE_0], x0[NAB];
#pragma unroll
          for (int e = 0; e < C::NE_0; ++e) e0[e] = XC[z + e * C::NCP + cp * C::ND + d];
          C::template bra_0<T>(e0, ABx, ABy, ABz, x0);
          gC[x] += C::template dot0<T>(Gam, x0);
          if constexpr (C::LC >= 1) {
            const int pw = C::CPOW[c][x];
            if (pw > 0) {
              const int cm = C::CMINUS[c][x];
#pragma unroll
              for (int e = 0; e < C::NE_0; ++e)
                e0[e] = XV[z + (C::U_EB + e) * C::NCM + cm * C::ND + d];
              C::template bra_0<T>(e0, ABx, ABy, ABz, x0);
              gC[x] -= pw * C::template dot0<T>(Gam, x0);
            }
          }
        }
      }
      const int o3 = m * g.n_atoms * 3;
#pragma unroll
      for (int x = 0; x < 3; ++x) {
        // partial sums of this lane's (c, d) share; C and D need the quartet's sum
        const double ga = fq * gA[x], gb = fq * gB[x];
        const double gc = fq * group_sum<GL>(gC[x]);
        const double gd = -(group_sum<GL>(ga + gb) + gc);
        const double sa = wave_sum(ga), sb = wave_sum(gb);
        if (lane == kWaveSumLane) {
          grad_add(lds, g.dEdR, o3 + atA * 3 + x, sa, det, nl);
          grad_add(lds, g.dEdR, o3 + atB * 3 + x, sb, det, nl);
        }
        if (active) {
          grad_add(lds, g.dEdR, o3 + atC * 3 + x, gc, det, nl);
          grad_add(lds, g.dEdR, o3 + atD * 3 + x, gd, det, nl);
        }
      }
    }
  }
  }
  if (lds) {
    __syncthreads();
    if (det == 0) {
      for (int t = threadIdx.x; t < nl; t += kBlock)
        if (gacc[t] != 0.0) atomic_add(&g.dEdR[t], gacc[t], 0);
    } else {
      const unsigned long long* wl = reinterpret_cast<const unsigned long long*>(gacc);
      unsigned long long* wg = reinterpret_cast<unsigned long long*>(g.dEdR);
      for (int t = threadIdx.x; t < nl; t += kBlock) {
        if (wl[t] != 0) atomicAdd(&wg[t], wl[t]);
        if (wl[t + nl] != 0) atomicAdd(&wg[t + det], wl[t + nl]);
      }
    }
  }
}

void launch_grad(int cls, int fp32, const GradLaunch& a, hipStream_t s);
int grad_ws_elems(int cls);
int grad_lanes(int cls);
int grad_lane_mask(int cls);

}  // namespace jk
