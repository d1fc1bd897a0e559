// hr_batch.h -- host side of batched execution, shared by the batch entry
// points and the server: one BatchSlot is the device state of one batch in
// flight (stream, table, workspace, captured graph).
#pragma once
#include <vector>

#include "hr_runtime.h"

namespace hr {
namespace rt {

struct BatchItem {
  QueryPlan plan;
  const double* theta = nullptr;   // host, n doubles (copied into the table)
  const double* v = nullptr;       // host, n doubles for the HVP kinds
  double* out = nullptr;           // host destination (nullptr: not copied out)
  bool zero = false;               // HVP with v = 0: result 0, no device work
  size_t ws_off = 0;               // workspace offset within the slot
  size_t out_off = 0;              // output offset within the table (doubles)
  uint64_t ticket = 0;             // server bookkeeping
};

struct BatchSlot {
  hr_ctx* ctx = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  int cus = 1, phase_blocks = 1;
  int raster_blocks[kRasterClasses] = {};   // persistent blocks per raster class
  int pt_blocks[3] = {1, 1, 1};    // per renders-per-draw class (1, 2, 4)
  uint64_t raster_class_items[kRasterClasses] = {};   // work items per class
  uint64_t pt_class_items[3] = {};
  void* dev = nullptr;             // device table: header, queries, task lists,
  void* host = nullptr;            //   queue segments, counters, theta/v, outputs
  size_t table_bytes = 0;          //   (pinned host mirror of the same layout)
  void* ws = nullptr;              // query workspaces, back to back
  size_t ws_bytes = 0;
  hipGraphExec_t exec = nullptr;   // the captured launch sequence
  size_t exec_lds = 0, exec_lds_pair = 0, exec_lds_pair32 = 0;
  unsigned exec_classes = 0;       // render classes launched by the captured sequence
  size_t lds = 0;                  // dynamic LDS of the persistent rasteriser
  size_t lds_pair = 0;             // and of its render-pair classes (64-disk layout,
  size_t lds_pair32 = 0;           //   32-disk layout)
  size_t class_lds(int c) const {
    return !raster_is_pair_class(c) ? lds : (c >= raster_pair_class(1, 32) ? lds_pair32 : lds_pair);
  }
  bool graph_used = false;
  bool allow_timing = true;        // phase timers (batch entry point only)
  int nq_ = 0;
  size_t upload_bytes_ = 0, out_off_ = 0, out_doubles_ = 0;
  uint64_t raster_items_ = 0, pt_items_ = 0;
  // A batch of one query runs the per-query kernels on this slot's stream and
  // workspace (the same bits as the batch kernels; no task lists, no queues).
  bool single_ = false;
  QueryPlan single_plan_{};
  QueryBufs single_bufs_{};
  const double* single_theta_ = nullptr;   // device pointers into the table
  const double* single_v_ = nullptr;
  double* single_out_ = nullptr;
  int single_S_ = 0, single_shape_ = 0;

  hr_status init(hr_ctx* c);
  void release();
  hr_status reserve_workspace(size_t bytes);
  hr_status reserve_table(size_t bytes);
  // lays out the table for `items` in the pinned mirror (sets ws_off/out_off)
  hr_status build(std::vector<BatchItem>& items);
  // upload, launch (graph replay or eager), download, record `done`; with
  // timing_ok false the launches are never timed, whatever the context says
  hr_status enqueue(bool use_graph, bool timing_ok = true);
  // copies each item's result from the pinned mirror to its destination
  void scatter(const std::vector<BatchItem>& items) const;
  void launches(hipStream_t st, bool time_phases);
  // render classes with work: raster classes in bits 0-11, path-traced in 16-18
  unsigned classes() const;
};

// validates one public query and plans it
hr_status plan_item(const hr_query& q, BatchItem* it);
// times raster samples-per-block and block shape for every untuned class of
// disk scene among `items`; the choice is kept in the context
hr_status autotune_raster(BatchSlot& slot, const std::vector<BatchItem>& items);

}  // namespace rt
}  // namespace hr
