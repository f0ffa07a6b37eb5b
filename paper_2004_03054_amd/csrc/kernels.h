// Kernel interfaces shared between the kernel sources and the host runtime.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "luda_internal.h"

namespace luda {

struct MergeTask {
  uint32_t a0, la, b0, lb;  // runs A and B as ranges of the source order array
  uint64_t out0;            // first output position
};

constexpr uint32_t SEG_C = 2048;  // items per segmentation chunk

struct SegJob {
  uint64_t base;     // first global item of the job
  uint32_t m;        // items of the job
  uint32_t chunk0;   // first chunk of the job
  uint32_t nchunks;
  uint32_t pad;
};

struct SegChunk {
  uint32_t job;
  uint32_t start, end;  // job-local item range
  uint32_t pad;
};

struct OutBlocks {
  uint64_t* s0;      // first survivor (global)
  uint32_t* cnt;     // entries
  uint32_t* size;    // contents bytes (trailer excluded)
  uint64_t* full;    // contents + 5
  uint32_t* job;
  uint32_t* file;
  uint64_t* off;     // offset inside its file
  uint32_t* ie_size; // bytes of its index block entry
};

struct OutFiles {
  uint32_t* job;
  uint64_t* b0;        // first output block
  uint32_t* nb;        // blocks
  uint64_t* data;      // data bytes (blocks + trailers)
  uint64_t* nwin;      // filter windows
  uint64_t* w0;        // first global filter window
  uint64_t* filter_off, *filter_size, *meta_off, *meta_size, *index_off, *index_size;
  uint64_t* size;      // whole file
  uint64_t* out;       // offset in the output buffer
  uint64_t* entries;
  uint64_t* keyr;      // 4 per file: smallest key offset (in the file) and length, largest key offset and length
};

// decode
struct WalkArgs {
  WalkSet ws;
  Inputs in;
  const uint8_t* ok;       // block passed its checksum
  const uint32_t* nr;      // restart count per block
  const uint64_t* ibase;   // first interval of each block
  const uint32_t* iblk;    // block of each interval
  const uint64_t* ni_dev;  // number of intervals
  uint32_t* icnt;          // count pass: entries per interval
  const uint64_t* ient;    // emit pass: first output of each interval
  WalkSet out_blk;         // index emit: the data block table
  const uint64_t* in_blk0; // index emit: first data block of each input
  Tuples tu;               // data emit: entry records
  uint32_t* maxklen;
  unsigned long long* err;
};
__global__ void k_footer(Inputs in, WalkSet idx, unsigned long long* err);
// compressed data blocks (type 1): staging room per block, then the second
// restart-count pass over the decompressed ones
constexpr uint64_t ZSTAGE_PAD = 64;  // readable bytes after each staged raw block
struct ZPass {
  uint64_t* cap;             // per block: staging bytes (0: not compressed); null for index blocks
  unsigned long long* tot;   // [0] compressed blocks, [1] staging bytes
  const uint8_t* ok;         // second pass: the block decompressed cleanly
  int only_z;                // second pass
};
__global__ void k_blk_nr(WalkSet ws, Inputs in, uint32_t* nr_out, unsigned long long* err, ZPass z);
// one wave per compressed data block: its Snappy stream into staging (at
// zoff), then the block table points at the raw bytes
__global__ void k_unsnappy(WalkSet ws, Inputs in, uint8_t* ok, const uint64_t* zcap, const uint64_t* zoff,
                           uint8_t* stage, unsigned long long* err);
__global__ void k_crc_wave(WalkSet ws, Inputs in, const uint32_t* g_crc, uint8_t* ok, unsigned long long* err,
                           unsigned long long* bytes_total);
// checksums of the inputs' index blocks against their trailers
// (at most cap index blocks; part and mseg as for k_crc_multi)
void launch_crc_index(WalkSet ws, Inputs in, const uint32_t* g_crc, uint8_t* ok, unsigned long long* err,
                      uint64_t cap, uint32_t* part, uint64_t* mseg, uint32_t grid, hipStream_t st);
__global__ void k_imap(WalkSet ws, const uint64_t* ibase, const uint64_t* ni_dev, uint32_t* iblk);
template <int KIND, int MODE>
__global__ void k_walk(WalkArgs A);
__global__ void k_keys(Tuples tu, WalkSet ws, Inputs in, uint32_t kw8, const uint64_t* n_dev, unsigned long long* err);
__global__ void k_order(Tuples tu, WalkSet ws, Inputs in, const uint64_t* in_e0, uint32_t kw8, const uint64_t* n_dev,
                        int32_t* in_cmp, unsigned long long* err);

// merge
__global__ void k_iota(uint32_t* idx, uint64_t n);
__global__ void k_fill_u32(uint32_t* p, uint32_t v, uint64_t n);
__global__ void k_fill_u64(unsigned long long* p, unsigned long long v, uint64_t n);
__global__ void k_merge(const MergeTask* tasks, uint32_t ntasks, const uint32_t* src, uint32_t* dst, Tuples tu,
                        uint32_t kw8, uint64_t total);
__global__ void k_dedup_flags(const uint32_t* ord, Tuples tu, uint32_t kw8, const JobDesc* jobs,
                              const uint64_t* snaps, const uint64_t* job_e0, uint32_t J, uint64_t n, uint32_t* keep,
                              unsigned long long* shadowed, unsigned long long* tomb, const uint32_t* active);
__global__ void k_scatter(const uint32_t* ord, const uint32_t* keep, const uint32_t* pos, uint64_t n,
                          uint32_t* surv);
// exclusive scan of n values (n from the device when n_dev is given; cap
// bounds it): out[0..n) and out[n] = total.  scratch holds cap/2048 + 2.
// Input values of type TI are summed as T.  Up to SCAN_ONE_MAX elements one
// workgroup does it in one launch.
constexpr uint64_t SCAN_ONE_MAX = 4096;
template <typename TI, typename T>
void launch_scan(const TI* in, uint64_t cap, const uint64_t* n_dev, T* out, T* scratch, hipStream_t st);
constexpr uint32_t MERGE_ITEMS_PER_THREAD = 8;

// plan
struct EncRec;
__global__ void k_prep(const uint32_t* surv, Tuples tu, uint32_t kw8, const uint64_t* job_s0, uint32_t J,
                       uint64_t S, uint32_t* sz_r, uint32_t* sz_n, uint32_t* shr, EncRec* rec);
struct BlockNext;
struct FileNext;
void launch_seg_exit_blocks(const SegChunk* ch, const uint32_t* nch_dev, uint32_t grid, const SegJob* sj,
                            const JobDesc* jobs, const uint32_t* sz_r, const uint32_t* sz_n, uint32_t* nxt,
                            uint32_t* ex, uint32_t* cnt, uint32_t* job_bmax, hipStream_t st);
void launch_seg_exit_files(const SegChunk* ch, const uint32_t* nch_dev, uint32_t grid, const SegJob* sj,
                           const JobDesc* jobs, const uint64_t* ob_excl, const uint64_t* ob_full, uint32_t* nxt,
                           uint32_t* ex, uint32_t* cnt, uint32_t* job_bmax, hipStream_t st);
__global__ void k_seg_compose(const SegJob* sj, uint32_t J, const uint32_t* ex, const uint32_t* cnt,
                              const uint32_t* job_bmax, uint32_t* chunk_entry, uint32_t* chunk_seg0,
                              uint32_t* job_nseg, uint32_t cap);
void launch_seg_mark(const SegChunk* ch, const uint32_t* nch_dev, uint32_t grid, const SegJob* sj,
                     const uint32_t* nxt, const uint32_t* chunk_entry, const uint32_t* chunk_seg0,
                     const uint64_t* job_seg_base, uint32_t* seg_first, hipStream_t st);
__global__ void k_make_segjobs(const uint64_t* base_excl, const uint32_t* counts, uint32_t J, SegJob* sj,
                               SegChunk* ch, uint32_t* nch_out);
__global__ void k_small_scan(const uint32_t* v, uint32_t J, uint64_t* out);
struct EntL;
__global__ void k_block_meta(const uint64_t* job_ob0, uint32_t J, const SegJob* sj_s, const JobDesc* jobs,
                             const uint32_t* seg_first, const uint32_t* sz_r, const uint32_t* sz_n,
                             const EncRec* rec, uint64_t cap, OutBlocks ob, uint32_t* ent_off, EntL* entl,
                             uint32_t* gapcnt);
__global__ void k_file_pre(const uint64_t* job_f0, uint32_t J, const uint64_t* job_ob0, const uint32_t* file_first,
                           const uint64_t* ob_excl, uint64_t cap, OutFiles of);
__global__ void k_block_post(const uint64_t* nfiles_total, OutFiles of, const uint64_t* ob_excl,
                             const uint64_t* job_ob0, uint32_t J, Tuples tu, const uint32_t* surv, uint64_t cap,
                             OutBlocks ob, uint32_t* win_keys, uint32_t* win_fb);
__global__ void k_win_size(const uint64_t* nwin_total, const uint64_t* file_w0_sorted, uint64_t nfiles,
                           OutFiles of, const JobDesc* jobs, const uint32_t* win_keys, uint64_t cap,
                           uint64_t* win_bytes, uint32_t* win_file, uint32_t* max_bytes);
__global__ void k_file_layout(const uint64_t* nfiles_total, OutFiles of, const uint64_t* win_off,
                              const uint64_t* ie_off, uint64_t cap);

// encode
// per survivor, written by k_prep for the encoder
struct EncRec {
  uint64_t vp;      // value address
  uint64_t tag;
  uint32_t e;       // decoded entry (key slot)
  uint32_t shared;  // key bytes shared with the previous survivor of its job
  uint32_t ulen;
  uint32_t vlen;
};
// per survivor, written by k_block_meta: the whole 16-byte chunks of its
// value in its block's chunk grid (chunks aligned to the end of the block
// message; chunk m covers message positions [16 m - gshift, 16 m - gshift +
// 16) with gshift = 16 ceil(n / 16) - n for a message of n bytes)
struct EntL {
  uint64_t vsrc;    // chunk m of the value interior is at vsrc + 16 m
  uint32_t ia;      // first chunk of the interior (also set when it is empty)
  uint32_t pieces;  // chunks of the interior
  uint32_t cum;     // interior chunks of the earlier entries of the block
  uint32_t pad;
};
// per output block, written by k_block_dst for the encoder
struct BlockRec {
  uint64_t dst;  // offset in the output buffer
  uint64_t s0;   // first survivor
  uint32_t cnt;
  uint32_t size;  // contents bytes (trailer excluded)
  uint32_t R;     // restart interval
  uint32_t pad;
};
// chunks per lane of the pipelined encoder: it takes blocks whose message
// (contents + type byte) is 16 to 64 * 16 * ENC_PIPE_CHUNKS bytes, of at most 64 entries
constexpr uint32_t ENC_PIPE_CHUNKS = 5;
__host__ __device__ constexpr bool enc_pipelined(uint32_t size, uint32_t cnt) {
  return size + 1 >= 16 && size + 1 <= 64 * 16 * ENC_PIPE_CHUNKS && cnt <= 64;
}
// big_list (optional): the ids of the blocks off the pipelined path, in any
// order, counted in big_n (room for big_cap: as many as the planning
// statistics counted; ids past it are not stored)
__global__ void k_block_dst(OutBlocks ob, OutFiles of, const JobDesc* jobs, const uint64_t* nblocks, uint64_t cap,
                            BlockRec* br, uint64_t* big_list, uint32_t* big_n, uint64_t big_cap);
struct EncodeArgs {
  const JobDesc* jobs;
  OutBlocks ob;
  OutFiles of;
  Tuples tu;
  const uint32_t* surv;
  const uint32_t* sz_r;
  const uint32_t* sz_n;
  const uint32_t* shr;
  const uint64_t* nblocks;  // device total of output blocks
  uint8_t* out;
  const uint32_t* g_crc;
  const uint32_t* ent_off;  // each survivor's entry offset inside its block
  const EncRec* rec;
  const BlockRec* blk;
  uint32_t kw8;
  const EntL* entl;         // each survivor's value interior in its block's chunk grid
  const uint64_t* gap_base; // first gap buffer slot of each block (and the total)
  uint4* gapbuf;            // gap chunks (16 bytes each)
};
// Gap chunks are written by groups of GAP_GROUP lanes per block, chunk by
// chunk, or entry-major by groups of GAP_EM_GROUP lanes (an LDS image of the
// block's gap slots) for blocks of GAP_EM_MIN to GAP_GROUP entries, at most
// GAP_SLOTS gap slots and keys of at most GAP_KW8 words
constexpr uint32_t GAP_GROUP = 16;
constexpr uint32_t GAP_SLOTS = 64;
constexpr uint32_t GAP_KW8 = 3;
constexpr uint32_t GAP_EM_MIN = 4;  // fewer entries leave most of a group's lanes idle
constexpr uint32_t GAP_EM_GROUP = 8;  // lanes per block in the entry-major form
__host__ __device__ constexpr bool gap_em_block(uint32_t cnt, uint32_t size, uint64_t slots) {
  return cnt <= GAP_GROUP && cnt >= GAP_EM_MIN && slots <= GAP_SLOTS && size + 1 >= 16;
}
template <bool EM>
__global__ void k_gaps(EncodeArgs A);  // EM: the entry-major blocks (and A.kw8 <= GAP_KW8), else the others
__global__ void k_encode(EncodeArgs A);
// the blocks k_encode leaves: those listed in list[0, nlist), or (list null)
// every block off the pipelined path
__global__ void k_encode_big(EncodeArgs A, const uint64_t* list, uint64_t nlist);
struct FilterArgs {
  const JobDesc* jobs;
  OutBlocks ob;
  OutFiles of;
  Tuples tu;
  const uint32_t* surv;
  const uint64_t* nwin;       // device total of windows
  const uint32_t* win_keys;
  const uint32_t* win_fb;
  const uint32_t* win_file;
  const uint64_t* win_bytes;
  const uint64_t* win_off;    // exclusive scan of win_bytes
  const uint64_t* hash;       // XXH64 of each survivor's user key
  uint8_t* out;
  uint32_t kw8;
  uint32_t lds_bytes;         // per wave
};
__global__ void k_key_hash(const uint32_t* surv, Tuples tu, uint32_t kw8, uint64_t n, uint64_t* hash);
__global__ void k_filter_small(FilterArgs A);
__global__ void k_filter(FilterArgs A);
__global__ void k_index_write(OutBlocks ob, OutFiles of, Tuples tu, const uint32_t* surv, const uint64_t* ie_off,
                              const uint64_t* nblocks, uint32_t kw8, uint64_t cap, uint8_t* out);
__global__ void k_meta(OutFiles of, const uint64_t* win_off, const uint64_t* nfiles, uint64_t cap, uint8_t* out);
__global__ void k_filter_offsets(OutFiles of, const uint64_t* nwin, const uint32_t* win_file,
                                 const uint64_t* win_off, uint64_t cap, uint8_t* out);
// misc
struct MailSegs {
  uint64_t src[12];
  uint32_t bytes[12];
  uint32_t dst[12];
  uint32_t n;
};
__global__ void k_mail(MailSegs m, uint8_t* mail);
// the readback's sequence number, written after k_mail into pinned memory
__global__ void k_mail_flag(uint64_t* flag, uint64_t seq);
struct UpSegs {
  uint64_t dst[16];
  uint32_t bytes[16];
  uint32_t src[16];
  uint32_t n;
};
__global__ void k_upload(UpSegs u, const uint8_t* up);
__global__ void k_gather_u64(const uint64_t* src, const uint64_t* idx, uint32_t n, uint64_t* out);
__global__ void k_ranges(const uint64_t* ient, const uint64_t* ibase, const uint64_t* blk0_of, uint32_t n,
                         uint64_t* out);
__global__ void k_job_surv(const uint64_t* job_e0, const uint32_t* kpos, uint32_t J, uint64_t* job_s0);
// stats: [0] largest block size, [1] most entries in a block, [2] a block
// under 16 bytes, [3] blocks off the pipelined encoder, [4] blocks whose
// gap chunks are written entry-major (gap_entry_major)
__global__ void k_plan_stats(OutBlocks ob, const uint64_t* job_ob0, uint32_t J, uint64_t cap,
                             const uint32_t* gapcnt, uint32_t* stats);
__global__ void k_file_entries(OutFiles of, OutBlocks ob, const uint32_t* surv, Tuples tu, const uint64_t* ie_off,
                               uint64_t nf, const uint8_t* ztype);
__global__ void k_ingest_max(const uint64_t* koff, uint64_t n, uint32_t* maxlen);
__global__ void k_ingest(const uint8_t* keys, const uint64_t* koff, const uint64_t* tags, const uint8_t* vals,
                         const uint64_t* voff, uint64_t n, Tuples tu, uint32_t kw8, uint32_t* surv);
__global__ void k_check_sorted(Tuples tu, uint32_t kw8, uint64_t n, uint32_t* bad);
// checksums of every file's filter, metaindex and index blocks (trailers
// written); part and mseg (3 cap + 1 slots) as for k_crc_multi
void launch_crc_files(OutFiles of, const uint64_t* nfiles, uint64_t cap, uint8_t* out, const uint32_t* g_crc,
                      uint32_t* part, uint64_t* mseg, uint32_t grid, hipStream_t st);

// compressed output blocks (k_snappy.hip)
__global__ void k_zprep(OutBlocks ob, const uint64_t* nblocks, uint64_t cap, uint32_t* zraw, uint64_t* zstride);
__global__ void k_block_dst_stage(OutBlocks ob, const uint64_t* zoff, const JobDesc* jobs, const uint64_t* nblocks,
                                  uint64_t cap, BlockRec* br);
__global__ void k_zsnappy(OutBlocks ob, const JobDesc* jobs, const uint64_t* nblocks, const uint8_t* stage,
                          const uint64_t* zoff, const uint32_t* zraw, uint8_t* zbuf, uint8_t* ztype);
__global__ void k_zplace(const BlockRec* br, const uint64_t* nblocks, const uint8_t* stage, const uint8_t* zbuf,
                         const uint64_t* zoff, const uint8_t* ztype, uint8_t* out);
void launch_crc_zblocks(const BlockRec* br, const uint64_t* nblocks, uint64_t cap, uint8_t* out, const uint32_t* g_crc,
                        uint32_t* part, uint64_t* mseg, uint32_t grid, hipStream_t st);
__global__ void k_zslots(OutFiles of, OutBlocks ob, const uint32_t* surv, Tuples tu, const uint8_t* ztype,
                         const uint64_t* nfiles, uint64_t cap, uint64_t* stride);
__global__ void k_zkeys(OutFiles of, OutBlocks ob, const uint32_t* surv, Tuples tu, const uint8_t* ztype,
                        uint32_t kw8, uint64_t nf, uint8_t* out);

}  // namespace luda
