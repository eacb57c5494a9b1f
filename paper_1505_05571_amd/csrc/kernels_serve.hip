// kernels_serve.hip -- one step of the serving loop: exact sums of a list of
// pieces of requests (gfx950).
//
// A piece is a range of one request's terms.  Pieces [0, nshort) are short
// and each is summed by one wavefront with the small-superaccumulator body;
// the others are summed one per workgroup with the large accumulator in
// carry mode (a step of short pieces only runs a lighter kernel of
// one-wavefront workgroups).  A request made of one piece is rounded where
// it is summed.  A request cut into several pieces (possibly over several
// steps) adds each piece into its accumulator slot with 64-bit atomics and
// takes a ticket; pieces of the step that completes the request carry the
// total piece count, and the piece whose ticket completes the count rounds
// (Discussion: add the small superaccumulators of the parts, round once).
// Steps run in stream order, so every piece of an earlier step has been
// added before any piece of a later one.
#include "exsum_blocks.h"
#include "exsum_internal.h"

namespace exsum {
namespace {

constexpr int kPieceCopies = 8;

template <int NW>
struct PieceShared {
  LargeShared L;
  long long wacc[NW][small_acc_words<kPieceCopies>()];
  unsigned long long wspec[NW][4];
};

// The step's piece list: in device memory, or (for a few pieces) in the
// kernel arguments, which saves a host-to-device copy at low load.
struct PieceTable {
  const Piece *p;
  __device__ Piece operator[](int i) const { return p[i]; }
};
struct InlinePieces {
  Piece p[kInlinePieces];
  __device__ Piece operator[](int i) const { return p[i]; }
};

template <int BLOCK, int VEC, int DEPTH, class Table>
__global__ __launch_bounds__(BLOCK) void piece_kernel(const Table P, int nshort, int np,
                                                      GlobalAcc *__restrict__ slots, int precombine) {
  constexpr int NW = BLOCK / 64;
  __shared__ PieceShared<NW> S;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // all lanes active here
  const int nlong = np - nshort;
  if (nlong > (int)blockIdx.x) large_init(S.L, tid, BLOCK);

  // short pieces: one per wavefront of the grid (a scalar loop counter)
  {
    long long *acc = S.wacc[wave];
    unsigned long long *spec = S.wspec[wave];
    for (int p = (int)blockIdx.x * NW + wave; p < nshort; p += (int)gridDim.x * NW) {
      const Piece pc = P[p];
      small_wave_zero<kPieceCopies>(acc, spec, lane);
      // a whole request (one piece) is rounded here and merged nowhere
      small_wave_accumulate<kPieceCopies>(acc, spec, SrcF64{pc.x}, 0, pc.n, lane, pc.expected == 1u);
      GlobalAcc *g = pc.expected == 1u ? nullptr : &slots[pc.slot];
      wave_merge_and_round(acc, spec, g, pc.expected, pc.out, lane);
    }
  }
  __syncthreads();

  // long pieces: each workgroup takes a contiguous run of the list.  Pieces
  // of one request lie next to each other in it (the scheduler gives the
  // oldest requests their pieces in a row) and share a slot and an expected
  // count, so a workgroup adds consecutive pieces of one request into its
  // large accumulator and flushes and merges once for all of them, the
  // ticket advancing by their number.  Every value that steers the loops
  // below is made wave-uniform (they hold workgroup barriers).
  const int nl = np - nshort;
  const int q0 = nshort + (int)((long long)nl * blockIdx.x / gridDim.x);
  const int q1 = nshort + (int)((long long)nl * (blockIdx.x + 1) / gridDim.x);
  const auto key_of = [&](int q, unsigned int &expected, int &slot) {
    const Piece pc = P[q];
    expected = (unsigned int)__builtin_amdgcn_readfirstlane((int)pc.expected);
    slot = __builtin_amdgcn_readfirstlane(pc.slot);
  };
  unsigned int tile = 0;
  for (int p = q0; p < q1;) {
    unsigned int expected;
    int slot;
    key_of(p, expected, slot);
    const Piece pc = P[p];
    int q = p;
    do {
      const Piece pq = P[q];
      accumulate_range<BLOCK, VEC, DEPTH, kCarryMode>(S.L, SrcF64{pq.x}, 0, pq.n, precombine, tile);
      q++;
      if (expected == 1u || q >= q1) break;
      unsigned int e2;
      int s2;
      key_of(q, e2, s2);
      if (e2 != expected || s2 != slot) break;
    } while (true);
    final_flush<BLOCK, true, kCarryMode>(S.L);
    GlobalAcc *g = expected == 1u ? nullptr : &slots[slot];
    merge_and_round(S.L.small, S.L.spec, &S.L.ticket, g, expected, pc.out, (unsigned int)(q - p));
    if (tid < 68) S.L.small[tid] = 0;
    if (tid < 3) S.L.spec[tid] = 0ull;
    __syncthreads();
    p = q;
  }
}

// A step whose pieces are all short (the common case at light load): one
// wavefront per workgroup and per piece, with only that wave's small
// accumulator in LDS, so a step of one short request costs what a single
// short sum costs.  The accumulator is cleared under the first loads of each
// piece.
template <class Table>
__global__ __launch_bounds__(64) void piece_short_kernel(const Table P, int nshort, GlobalAcc *__restrict__ slots) {
  __shared__ long long acc[small_acc_words<kPieceCopies>()];
  __shared__ unsigned long long spec[4];
  const int lane = threadIdx.x;
  for (int p = (int)blockIdx.x; p < nshort; p += (int)gridDim.x) {
    const Piece pc = P[p];
    small_wave_accumulate<kPieceCopies, SrcF64, true>(acc, spec, SrcF64{pc.x}, 0, pc.n, lane, pc.expected == 1u);
    GlobalAcc *g = pc.expected == 1u ? nullptr : &slots[pc.slot];
    wave_merge_and_round(acc, spec, g, pc.expected, pc.out, lane);
  }
}

constexpr int kPieceBlock = 512;
constexpr int kShortStepGrid = 4096;     // workgroups of the short-only step kernel at most

}  // namespace

hipError_t launch_pieces(const Piece *pieces, const Piece *host_pieces, int nshort, int npieces, GlobalAcc *slots,
                         hipStream_t s, int grid, int precombine) {
  if (npieces <= 0) return hipSuccess;
  if (grid < 1) grid = 1;
  if (nshort == npieces) {
    const int g = npieces < kShortStepGrid ? npieces : kShortStepGrid;
    if (host_pieces != nullptr && npieces <= kInlinePieces) {
      InlinePieces t;
      for (int i = 0; i < kInlinePieces; i++) t.p[i] = i < npieces ? host_pieces[i] : Piece{nullptr, 0, nullptr, 0, 0u};
      hipLaunchKernelGGL((piece_short_kernel<InlinePieces>), dim3(g), dim3(64), 0, s, t, nshort, slots);
    } else {
      hipLaunchKernelGGL((piece_short_kernel<PieceTable>), dim3(g), dim3(64), 0, s, PieceTable{pieces}, nshort,
                         slots);
    }
    return hipGetLastError();
  }
  if (host_pieces != nullptr && npieces <= kInlinePieces) {
    InlinePieces t;
    for (int i = 0; i < kInlinePieces; i++) t.p[i] = i < npieces ? host_pieces[i] : Piece{nullptr, 0, nullptr, 0, 0u};
    hipLaunchKernelGGL((piece_kernel<kPieceBlock, 4, 2, InlinePieces>), dim3(grid), dim3(kPieceBlock), 0, s, t,
                       nshort, npieces, slots, precombine);
  } else {
    hipLaunchKernelGGL((piece_kernel<kPieceBlock, 4, 2, PieceTable>), dim3(grid), dim3(kPieceBlock), 0, s,
                       PieceTable{pieces}, nshort, npieces, slots, precombine);
  }
  return hipGetLastError();
}

int pieces_block() { return kPieceBlock; }

}  // namespace exsum
