// Round driver shared by the single-scene and the batched entry points.
#pragma once
#include <string>
#include <vector>

#include "../../include/nanogs.h"
#include "internal.h"

namespace ng {

// Working layout of the splats (see internal.h for the fields).
struct Work {
  float4* cen;
  int* lg;
  float4* shp;
  float* sh;
  int* org;
  int* sg;  // segment (job position) of each row
};

// Options read from nanogs_options.
struct Opts {
  int S = 1;
  int app_dims = NG_SH;
  int precision = NANOGS_PREC_FP32;
  float fb_ratio = 1.0f / 256.0f;
  uint64_t seed = 0;
  int max_rounds = 0;
  int* d_trace = nullptr;
  int* d_origin = nullptr;
  int timing = 0;
  float tau = -1.0f;  // opacity pre-filter threshold (< 0: off)
  int cost_mode = NANOGS_COST_MC;
  int refresh = NANOGS_REFRESH_FULL;
  float pass_frac = 0.0f;  // per-pass pair cap (0: none)
};

enum JobState { JOB_QUEUED = 0, JOB_RUNNING = 1, JOB_DRAINING = 2, JOB_DONE = 3, JOB_FAILED = 4 };

struct JobSpec {
  nanogs_gaussians in;   // device, stored form, n rows
  nanogs_gaussians out;  // device, stored form, capacity n
  long long n = 0;
  long long target = 1;
  int k = 16;
  uint64_t seed = 0;
  int* d_origin = nullptr;  // nullable device [n]
  int* d_trace = nullptr;   // nullable device [n][2] (single-job batches only)
  // coarse-to-fine hierarchy (single-job batches only): each pass's set in
  // the stored form at rows lod_offsets[r].. of lod, and lod_parent[row] =
  // index of the splat of the next level it becomes
  nanogs_gaussians lod = {nullptr, nullptr, nullptr, nullptr, nullptr};
  int* lod_parent = nullptr;
  long long lod_cap = 0;
  long long* lod_offsets = nullptr;  // host [NANOGS_MAX_ROUNDS + 1]
};

struct Job {
  JobSpec spec;
  int id = -1;
  int state = JOB_QUEUED;
  int status = NANOGS_OK;
  std::string error;
  long long N = 0;     // current count
  long long row0 = 0;  // first row (and logical index) in the working set
  int round = 0;
  long long traced = 0;
  int lod_levels = 0;  // hierarchy levels written
  long long lod_used = 0;
  long long prev_n = 0;  // rows of the last pass that merged (local refresh)
  int prev_keff = 0;
  unsigned box[6] = {0, 0, 0, 0, 0, 0};
  nanogs_stats stats;
};

struct EngineWs;

// A working set of at most `rows` rows and `jobs` scenes, kNN size <= kmax,
// carved from a caller workspace of workspace_bytes(rows, kmax, jobs).
class Engine {
 public:
  static size_t workspace_bytes(long long rows, int kmax, int jobs);
  Engine(long long rows, int kmax, int jobs, const Opts& o, void* ws, hipStream_t st);
  ~Engine();
  Engine(const Engine&) = delete;
  Engine& operator=(const Engine&) = delete;

  int submit(const JobSpec& spec);  // returns the job id
  // Cancels a queued or running job (state FAILED, status ECANCELLED; a
  // running job's rows leave the working set at the next pass and its output
  // is not written).  Returns false if the job had already finished.
  bool cancel(int id);
  // One pass for every live job (queued jobs join first if they fit).
  // Returns the number of jobs that completed (or failed) in this step.
  int step(StageTimer* T = nullptr);
  void run(StageTimer* T = nullptr);  // steps until every job is done
  bool idle() const;
  long long rows_in_use() const;
  long long capacity() const { return R_; }
  const Job& job(int id) const { return jobs_[id]; }
  int num_jobs() const { return (int)jobs_.size(); }
  void set_stream(hipStream_t st) { st_ = st; }

 private:
  bool setup_job(Job& j, int pos);
  void finish_job(Job& j, const Work& w);

  long long R_;
  int K_, J_;
  // page-locked host memory: per-pass uploads (segment table, draws,
  // budgets) and the readback of the pass's counts after its one
  // synchronisation
  char* stage_ = nullptr;
  long long* hb_ = nullptr;
  Opts o_;
  hipStream_t st_;
  EngineWs* W_;
  int cur_ = 0;
  long long Ntot_ = 0;
  std::vector<Job> jobs_;
  std::vector<int> queue_;  // job ids waiting for rows
  std::vector<int> live_;   // job ids with rows in the working set, in row order
};

}  // namespace ng
