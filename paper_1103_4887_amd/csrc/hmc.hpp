// Hybrid Monte Carlo: kernel arguments and launcher.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.hpp"

namespace pimc {

constexpr int HMC_BLOCK = 256;  // sites per block of the leapfrog kernels

struct HmcArgs {
  ModelArgs m;
  Consts<float> cf;
  Consts<double> cd;
  int32_t B;               // chains (windows)
  int32_t nblocks;         // blocks of HMC_BLOCK sites over all chains
  const int64_t* offsets;  // device [B+1] packed site offsets
  const int32_t* bmap;     // device [nblocks] -> chain
  const int32_t* bfirst;   // device [B+1] first block of each chain
  void* X;                 // [S][4] positions (path precision), in/out
  double* p;               // [B][7] parameters, in/out
  const void* y;
  const void* I;
  const uint32_t* chain;   // [B] Philox chain ids
  uint64_t seed;
  uint64_t* kptr;          // device: proposal index of the next proposal
  uint64_t k_first;        // proposal index of the first proposal of the call
  double eps;              // leapfrog step
  double minv[11];         // inverse masses: (V, m, h, n) then p1..p7
  // workspace
  void* Q1;                // [S][4] positions, odd steps
  void* R0;                // [S][4] momenta, even half steps
  void* R1;                // [S][4] momenta, odd half steps
  void* X0;                // [S][4] start of the trajectory
  double* p0;              // [B][7]
  double* pbuf;            // [2][B][7] parameters by step parity
  double* rpbuf;           // [2][B][7] parameter momenta by step parity
  double* part;            // [2][nblocks][16] block partials by step parity
  double* H0;              // [B]
  uint32_t* outside;       // [B] a position left the box
  uint8_t* accepted;       // [B] decision of the last proposal
  double* dH;              // [B] H1 - H0 of the last proposal
  // statistics (nullable)
  int64_t* acc;            // [B][PIMC_NACC]
  double* ptrace;          // [B][ntrace][7]
  double* dHtrace;         // [B][ntrace]
  int64_t ntrace;
  // trajectory of the last proposal (nullable): after leapfrog kernel s,
  // positions q(s) and momenta r(s+1/2) (r(L) after the last) in
  // tq, tr [L+1][S][4] (path precision); p(s) in tp [L+1][B][7] and the
  // parameter momenta rp(0), rp(s-1/2) (s = 1..L), rp(L) in trp [L+2][B][7]
  void* tq;
  void* tr;
  double* tp;
  double* trp;
  int64_t S;               // packed sites of the batch
};

int launch_hmc_proposal(const HmcArgs& a, bool fp64, int L, hipStream_t s);

}  // namespace pimc
