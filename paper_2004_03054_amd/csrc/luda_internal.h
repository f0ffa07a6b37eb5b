// Internal data layout shared by the host orchestration and the kernels.
//
// All arrays are flat over a batch of jobs: global input index g, global data
// block index b, global decoded-entry index e, sorted position p, survivor
// index s, output block index ob, output file index f, filter window index w.
// Each job owns one contiguous range of every index space.
#pragma once
#include <stdint.h>

namespace luda {

enum ErrCode : uint32_t {
  EC_FORMAT = 1,
  EC_CHECKSUM = 2,
  EC_UNSUPPORTED = 3,
  EC_UNSORTED = 4,
  EC_LIMIT = 5,  // a size beyond what the GPU path supports
  EC_DEVICE = 6, // a bounded device wait gave up
};
enum Where : uint32_t { W_FOOTER = 0, W_INDEX = 1, W_DATA = 2 };
enum Phase : uint32_t { P_TRAILER = 0, P_RESTARTS = 1, P_ENTRIES = 2 };
// footer phases: 0 = file shorter than a footer (offset 0 of the file),
// 1 = offset relative to the footer start
enum FooterPhase : uint32_t { FP_SHORT = 0, FP_REL = 1 };

constexpr uint64_t ERR_NONE = ~0ull;
constexpr uint64_t TABLE_MAGIC = 0xdb4775248b80fb57ull;
constexpr uint32_t FILTER_BASE_LG = 11;
// bytes of one segment of a long block's checksum (one wave step)
constexpr uint32_t CRC_SEG_BYTES = 4096;

struct JobDesc {
  uint32_t block_size;
  uint32_t restart_interval;
  uint32_t bloom_bits_per_key;
  uint32_t bottommost;
  uint64_t target_file_size;
  uint32_t in_first;  // first global input
  uint32_t n_in;
  uint32_t snap_first;  // the job's live snapshots: [snap_first, snap_first + n_snap) of the call's list
  uint32_t n_snap;
  uint32_t compression;  // output data blocks: 0 raw, 1 Snappy when it saves an eighth
  uint32_t pad;
};

struct Inputs {
  const uint64_t* ptr;   // device address of each input table
  const uint64_t* size;  // bytes
  const uint32_t* job;   // owning job
  const uint32_t* local; // index inside its job
  uint32_t n;            // number of inputs
};

// A set of blocks to read: index blocks (one per input) or data blocks.
struct WalkSet {
  uint64_t* ptr;          // device address of the block contents
  uint32_t* size;         // contents bytes (trailer excluded)
  uint32_t* input;        // global input
  uint32_t* local;        // block number inside its input
  uint8_t* skip;          // 1: not read (its input already failed)
  const uint64_t* n_dev;  // number of blocks (device)
  uint32_t where;         // W_INDEX or W_DATA
};

// decoded entries (struct of arrays)
struct Tuples {
  uint64_t* kp0;   // user key bytes 0..7, big endian, zero padded
  uint64_t* kp1;   // user key bytes 8..15
  uint64_t* tag;
  uint32_t* ulen;  // user key length
  uint64_t* heap;  // user key slots, KW bytes each
  uint64_t* kd;    // device address of the entry's key delta
  uint64_t* sn;    // shared | non_shared << 32
  uint64_t* vp;    // device address of the value
  uint32_t* vlen;
  uint32_t* blk;   // data block
  uint32_t* eoff;  // entry offset inside the block contents
};

}  // namespace luda
