// Device view of a factor in the chunk-sliced layout used by the triangular
// solves (shared by the kernels and the host code that builds it).
#pragma once

namespace pmg {

// Off-chunk slots are gathered in batches of this many per lane.
constexpr int kTriBatch = 32;
// Slot widths are rounded up to this; column indices load in groups of it.
constexpr int kColGroup = 4;
// Padding entries at the end of each sliced array (one 16-byte group per lane).
constexpr int kTriPad = 64 * kColGroup;
// Ticket counters of one solve: the ticket counter, then kTicketStride words
// (128 bytes) further the count of exited waves; kTicketWords words per
// solve.  Every wave of the grid draws its tickets from the one counter, so
// tickets are handed out in the order waves ask for them, whichever waves
// are resident.
constexpr int kTicketStride = 32;
constexpr int kTicketWords = 2 * kTicketStride;
// Words of a workspace's solve state: the lower solve's counters, the upper
// solve's, then the fault word (TriCtl) shared by both.
constexpr int kTicketAlloc = 2 * kTicketWords + kTicketStride;
// Default bound on the polls of one wave waiting for one batch of entries
// (each poll sleeps ~128 cycles and reloads the pending entries, so the bound
// is seconds, far above any wait of a correct schedule).  A wave that reaches
// it sets the solve's fault word and stops waiting; every other wave stops
// waiting once it sees the word, so the grid always drains.
constexpr int kPollLimit = 1 << 22;

// Marker of a solution entry that is not final yet.  Before a triangular
// solve the output vector is filled with it; a wave that needs an entry
// reloads it until the marker is gone, so the values themselves carry the
// readiness and no flags or fences are needed.  Both are signalling NaNs,
// which no arithmetic produces (results are quiet NaNs at worst), and a
// stored value with the marker's bits is replaced by the canonical quiet NaN.
constexpr unsigned long long kPending64 = 0x7FF0DEAD0000DEADull;
constexpr unsigned kPending32 = 0x7F80DEADu;

// Factors in the chunk-sliced layout of the triangular solves.  A chunk is
// up to 64 consecutive rows of one segment, lane = row - chunk start; q is
// the chunk's natural index (chunks numbered by first row).  Chunks are taken
// in a topological order of the chunk dependency graph, by level, so a wave
// only ever waits for chunks taken before its own.
//   Off-chunk entries: slot u of lane l, u < off_w[q], per row sorted by the
//   level of the chunk holding the source row (ties: lower factor ascending
//   columns, upper descending), so entries that are final early come first.
//   Each row's entries fill its last slots (right-aligned) and padding,
//   column -1 and value 0, the first ones, so the entries every row waits
//   for longest share the last slots.
//   In-chunk entries: slot u of lane l, u < in_w[q], the position j of the
//   source row inside the chunk (-1 for padding) and the value.  For the
//   upper factor the value is divided by the diagonal of its column,
//   U_ij / U_jj, so the in-chunk recurrence runs on undivided partial sums
//   and each row is divided by its own diagonal once at the end.
// Slot widths are multiples of kColGroup, so every chunk starts at a
// multiple of 64 * kColGroup entries.  On the host (and in exports) slot u of
// lane l sits at ptr[q] + 64 u + l.  On the device each lane's slots come in
// 16-byte groups, one vector load each: columns in groups of kColGroup = 4 at
// ptr[q] + 64 u + 4 l + u % 4 (u a multiple of 4 for the group's first), values
// in groups of G = 16 / sizeof(T) at ptr[q] + 64 u + G l + u % G.  A wave's
// load of one group is 1 KiB contiguous, and a batch of kTriBatch slots takes
// kTriBatch / 4 + kTriBatch / G loads besides its gathers, which keeps a
// batch's loads within the 63 a wave can have outstanding.  Padding columns
// are stored as n on the device: gathers address the solution vector through
// a buffer resource of n entries, whose range check returns 0 for them.  The arrays end
// with kTriPad padding entries (column -1, value 0) at off_pad and in_pad,
// one group per lane, which lanes without an entry load instead, so every
// load is unconditional and its value needs no select.
//
// The per-chunk scalars are packed in ticket order, one 32-byte record per
// ticket, so a wave reads all of them with one scalar load.
struct alignas(32) TriMeta {
  int row0, nrow;      // first row and rows of the chunk
  int off_ptr, off_w;  // off-chunk slots
  int in_ptr, in_w;    // in-chunk slots
  int unused[2];
};

template <typename T>
struct TriDev {
  int off_pad, in_pad;
  int n;                // rows of the factor; the device's off_col holds n for padding
                        // (the host arrays and exports hold -1)
  const TriMeta* meta;  // by ticket
  const int* off_col;
  const T* off_val;
  const int* in_j;
  const T* in_val;
  const T* diag;  // upper factor only
};

}  // namespace pmg
