// Device-side data layout shared by the HIP kernels and the host driver of
// libgridplan.  Everything lives in flat arrays; per-scenario and
// per-network descriptors give offsets into them.
#pragma once
#include <stdint.h>

namespace gp {

constexpr int kStats = 15;  // FP64 statistics per tile / per scenario

// statistic slots (sums unless noted)
enum Stat {
  ST_RES_MAX = 0,   // max |E x - e| over balance rows   (max-reduced)
  ST_DUAL_MAX = 1,  // max |(E'y - q - r x)| over free entries (max-reduced)
  ST_XMAX = 2,      // max |x|                           (max-reduced)
  ST_RESF_MAX = 3,  // max |E x - e| over flow rows      (max-reduced)
  ST_RESS_MAX = 4,  // max |E x - e| over SOC and ramp rows (max-reduced)
  ST_P = 5,         // (r/2)||x||^2 + q'x
  ST_D = 6,         // dual function value
  ST_DX2 = 7,       // sum rho_i (xhat - x0)^2
  ST_DY2 = 8,       // sum rowden (yhat - y0)^2
  ST_EMIS = 9,      // sum emis_g p
  ST_FUEL = 10,     // sum cost_g p
  ST_RES2 = 11,     // sum (E x - e)^2 over all rows
  ST_DUAL2 = 12,    // sum (E'y - q - r x)^2 over free entries
  ST_D0 = 13,       // dual function at y = 0 (its box terms): the objective's
                    // scale when the optimum is near zero (adjoint solves)
  ST_PD = 14,       // sum load * pi over balance rows (dispatch solve)
};
constexpr int kMaxStats = 5;  // slots [0, kMaxStats) are maxima, the rest sums

// work classes of the primal (variable) sweep
enum VarClass { VC_GEN = 0, VC_LINE = 1, VC_NODE = 2, VC_BATT = 3, VC_RAMP = 4 };
// work classes of the dual (row) sweep
enum RowClass { RC_BAL = 0, RC_FLOW = 1, RC_SOC = 2, RC_RAMP = 3 };
// work-queue counters: one per XCD, kQueueStride u64 words apart; a sweep
// uses kQueueWords words (dual sweep first, then the primal sweep)
constexpr int kXcd = 8;
constexpr int kQueueStride = 16;
constexpr int kQueueWords = kXcd * kQueueStride;
enum ResetMode { RESET_WARM = 0, RESET_COLD = 1, RESET_PROBE = 2, RESET_RESTORE = 3 };

// a sweep tile whose scenario has T divisible by 4 is processed four hours
// per thread (16-byte loads of the FP32 state, 32-byte runs of the duals)
constexpr int32_t kTileVec4 = 0x100;

struct Tile {
  int32_t scen;   // scenario index
  int32_t cls;    // VarClass or RowClass (sweep tables: | kTileVec4)
  int32_t start;  // first local item (VC_* / RC_BAL / RC_FLOW) or battery index (RC_SOC)
  int32_t count;  // items in this tile (RC_SOC: chains; one per block unless four hours per thread)
};

struct ScenDev {
  int32_t net;       // network index
  int32_t T;         // hours
  int64_t xoff;      // offset of the scenario's x block
  int64_t yoff;      // offset of the scenario's y block
  int64_t aoff;      // offset of avail [G*T]
  int64_t doff;      // offset of load [N*T]
  int32_t tap_off;   // offset of the SOC-chain circulant taps
  int32_t ntap;      // taps h_0..h_{ntap-1} (symmetric, |j| < ntap)
};

struct NetDev {
  int32_t N, L, G, B;
  int32_t gen_off;   // into gen_* arrays
  int32_t line_off;  // into line_* arrays
  int32_t node_off;  // into node arrays (sig_bal, rho_th, rowden_bal)
  int32_t batt_off;  // into batt_node
  int32_t tptr_off;  // into term_ptr (N+1 entries)
  int32_t aptr_off;  // into ang_ptr (N+1 entries)
  int32_t eta_off;   // into eta (K_net entries: gens, lines, batteries)
  int32_t Lac;       // AC lines [0, Lac) have a flow row; lines [Lac, L) are
                     // HVDC links: their flow-row slots stay zero, and their
                     // susceptance is stored as 0 so no angle sees them
  int32_t R;         // ramp-limited generators (ramp variables s [R][T] after
                     // u in x, ramp rows [R][T] after the SOC rows in y)
  int32_t ramp_off;  // into ramp_gen / ramp_rho
};

// terminal codes of the nodal-balance CSR: (index << 2) | type
enum TermType { TT_GEN = 0, TT_BATT = 1, TT_LINE_TO = 2, TT_LINE_FROM = 3 };

struct Weights {
  float wb;     // balance-copy weight (generators, battery ch/dis, line ends)
  float wu;     // balance-copy weight of unserved load
  float wf;     // flow-row copy weight of the line flow
  float wth;    // flow-row copy weight of an angle, per beta^2
  float ws;     // SOC-chain copy weight
  float sig_flow;  // 1 / (1/wf + 2/wth)
  float rho_f;  // 2 wb + wf
  float rho_b;  // wb + ws  (ch, dis)
};

struct Args {
  // geometry
  const ScenDev* scen;
  const NetDev* net;
  const Tile* vtiles;  // variable tiles, one item per thread (checks, resets, masks)
  const Tile* rtiles;  // row tiles, one item per thread
  int32_t nvt, nrt;
  const Tile* svt;     // tiles of the two sweeps (four hours per thread where
  const Tile* srt;     // the scenario allows it)
  int32_t nsvt, nsrt;
  int32_t mode;        // 0 dispatch, 1 adjoint (active entries fixed, free elsewhere)
  int32_t qgrab;       // work-queue form: tiles taken per counter update
  // network data
  const int32_t* gen_node;
  const float* gen_cost;
  const float* gen_emis;
  const int32_t* line_from;
  const int32_t* line_to;
  const float* line_beta;   // susceptance at the current capacities (0 for HVDC links)
  const float* line_dbeta;  // d beta_l / d eta_l (0 unless the line's susceptance scales)
  const int32_t* batt_node;
  const int32_t* term_ptr;
  const int32_t* term;
  const int32_t* ang_ptr;
  const int32_t* ang;
  const float* sig_bal;     // per node: 1 / sum_j a_j^2 / w_j over the balance row
  const float* rho_th;      // per node: wth * sum of incident beta^2
  const float* taps;        // SOC circulant inverse taps (unscaled by primal weight)
  // scenario data
  const float* avail;
  const float* load;
  const float* eta;         // capacities (FP32)
  // state
  float* x;       // primal state, FP32
  float* x0;      // its anchor
  float* xhat;
  // Duals.  The anchor y0 and the output yhat are FP64: prices reach the
  // unserved-load penalty while the primal update needs E'y - q to far
  // better than FP32 resolution there.  The iterate is held as an FP32
  // offset from the anchor: dbar = ybar - y0, the extrapolated dual
  // 2 yhat - y of the last row sweep; the next Halpern iterate is
  // y0 + lambda * dbar.  Offsets stay small between restarts (the anchor
  // moves to the output point at each), so FP32 resolves them.
  double* y0;
  float* dbar;
  double* yhat;
  const uint8_t* amask;     // adjoint mode: 1 = entry held at its bound
  // per-scenario control
  const float* cw;          // primal weight
  const float* cwf;         // flow-class weight multiplier (flow rows and angles)
  const int32_t* kbase;     // Halpern inner counter at the start of the chunk
  const int32_t* active;    // 1 = iterate this scenario
  const int32_t* restart;   // 1 = restart from (xhat, yhat) (restart kernel only)
  // constants
  float r, lambda_u, eff, hours;
  float omega;              // adjoint mode: emission weight
  Weights w;
  // statistics
  double* part_v;           // [nvt][kStats]
  double* part_r;           // [nrt][kStats]
  const int32_t* ranges;    // [nb][4]: first/last variable tile, first/last row tile
  const int32_t* bscen;     // [nb] scenario of each batch entry
  double* stats;            // [nb][kStats]
  // (fields below are used by ramp-limited networks and price objectives
  // only; they sit last so the sweeps' common fields keep their offsets)
  const int32_t* gen_ramp;  // per generator: its ramp index (network-local) or -1
  const int32_t* ramp_gen;  // per ramp index: the generator (network-local)
  const float* ramp_rho;    // per ramp index: share of capacity per hour
  float lmp;                // adjoint mode: weight of sum pi D in the planner
                            // objective (the adjoint's balance rows carry lmp D)
  float wr;                 // ramp-row copy weight of a generator output (two per output)
  float wsr;                // ramp-row copy weight of a ramp variable
  float sig_ramp;           // 1 / (2/wr + 1/wsr): the ramp rows' dual step
};

}  // namespace gp
