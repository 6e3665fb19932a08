// Host-side objects of libsgweno (plans, solvers, batches).
#pragma once

#include <array>
#include <vector>

#include "sgw_internal.h"

struct sgw_plan {
    sgw_problem pb;
    sgw_config cfg;
    int G = 0;
    int N = 0;                                 // finest nodes per direction
    int64_t fine_nodes = 0;
    int64_t total_nodes = 0;
    int64_t nitems = 0;                        // stage boxes over all grids
    int64_t nitems_whole = 0;                  // the first boxes of the list: grids that are one box
    size_t stage_lds = 0;                      // max LDS bytes of a box
    size_t lds_whole = 0, lds_boxed = 0;       // the same over the one-box grids and over the others
    std::vector<std::array<int, 4>> levels;
    std::vector<int> coefs;
    std::vector<int64_t> offsets;              // element offset of each grid in a state copy
    std::vector<GridDev> grids;                // geometry only (pointers filled by the solver)
    std::vector<int64_t> coef_off;             // [G][4] offsets into the coefficient tables
    int fine_T[SGW_MAX_DIM] = {1, 1, 1, 1};
    size_t pro_buf_elems = 0;                  // prolongation LDS buffer A (and B in the old form)
    size_t pro_bufb_elems = 0;                 // buffer B
    bool fine_lines = false;                   // 3D/4D line form of the prolongation
    bool line_mode = false;                    // the stage runs as line sweeps (no boxes): 4D, zero
                                               // boundary or relaxation
    bool relax = false;                        // relaxation source on
    bool vm = false;                           // Vlasov-Maxwell: fields per grid
    uint64_t fields_off = 0;                   // byte offset of the fields in a state copy
    int64_t fields_total = 0;                  // field values over all grids (3 n_1 each)
    int zmask = 0;                             // bit k: zero boundary in direction k
    bool plane01 = false;                      // 4D: directions 1 and 2 in one plane launch per stage
    int64_t nplane_items = 0;                  // its work items over all grids
    int64_t nrho_items = 0;                    // density first-pass work items over all grids
    int64_t nrho_final = 0;                    // density second-pass work items (column blocks)
    std::vector<int64_t> mu_off;               // [G][4] offsets into the velocity factor tables
    size_t pro_rows_max = 0;                   // its LDS row-offset table entries
    size_t pro_lds = 0;                        // LDS bytes of a prolongation workgroup
    uint64_t copy_bytes = 0, state_bytes = 0, scratch_bytes = 0;
    uint64_t off_grids = 0, off_req = 0, off_items = 0, off_alpha = 0, off_coef = 0, off_coef_off = 0;
    uint64_t off_pro = 0, off_fine = 0, off_partials = 0, off_result = 0, off_foot = 0, off_stab = 0;
    uint64_t off_mu = 0, off_rho = 0, off_rho_part = 0, off_rho_items = 0, off_vm_alpha = 0, off_plane_items = 0;
};

struct sgw_solver {
    sgw_plan* plan = nullptr;
    unsigned char* state = nullptr;
    unsigned char* scratch = nullptr;
    hipStream_t stream = nullptr;
    GridDev* grids_d = nullptr;
    ReqDev* req_d = nullptr;
    WorkItem* items_d = nullptr;
    unsigned long long* alpha_d = nullptr;
    double* coef_d = nullptr;
    int64_t* coef_off_d = nullptr;
    ProDev* pro_d = nullptr;
    FineDev* fine_d = nullptr;
    double* partials_d = nullptr;
    double* result_d = nullptr;
    double* foot_d = nullptr;
    RhoItem* rho_items_d = nullptr;
    WorkItem* plane_items_d = nullptr;
    std::vector<int> plane_first;              // first plane item of each grid (G + 1 entries)
    std::vector<GridDev> grids_h;
    std::vector<WorkItem> items_h;
    std::vector<ProDev> pro_h;
    FineDev fine_h;
    std::vector<unsigned char> stab_h;         // prolongation coefficient table (host copy of the upload)
    ReqDev req_h;
    ReqDev* req_pinned = nullptr;
    bool restricted = false;
    double t_host = 0.0;
    int grid = 1;                              // workgroups of a persistent stage launch
    int grid_whole = 1;                        // the same for the three-stage launch of one-box grids
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    int graph_steps = 0;
    int batch_slot = -1;
};

sgw_status sgw_fail(sgw_status st, const char* fmt, ...);
sgw_status sgw_hip_fail(hipError_t e, const char* what);

// Pinned staging buffers for host-to-device list uploads (staging.hip): acquire a
// buffer of at least `bytes`, fill it, upload parts of it in stream order, then
// release it behind the copies (an event, no host wait).
hipError_t staging_acquire(size_t bytes, int* handle, void** host);
hipError_t staging_upload(int handle, size_t offset, void* dst_dev, size_t bytes, hipStream_t s);
hipError_t staging_release(int handle, hipStream_t s);
void staging_cancel(int handle);  // nothing was uploaded from it

struct Staging {
    int handle = -1;
    unsigned char* host = nullptr;
    hipError_t err = hipSuccess;
    hipStream_t stream = nullptr;
    bool uploaded = false;
    explicit Staging(size_t bytes)
    {
        void* p = nullptr;
        err = staging_acquire(bytes ? bytes : 1, &handle, &p);
        host = (unsigned char*)p;
        if (err != hipSuccess) handle = -1;
    }
    // every upload from one buffer goes to one stream: the release event is recorded there
    hipError_t upload(size_t offset, void* dst_dev, size_t bytes, hipStream_t s)
    {
        if (handle < 0) return err != hipSuccess ? err : hipErrorInvalidValue;
        if (uploaded && s != stream) return hipErrorInvalidValue;
        stream = s;
        uploaded = true;
        return staging_upload(handle, offset, dst_dev, bytes, s);
    }
    // the buffer returns to the pool once the copies enqueued so far have run
    ~Staging()
    {
        if (handle < 0) return;
        if (uploaded)
            (void)staging_release(handle, stream);
        else
            staging_cancel(handle);
    }
    Staging(const Staging&) = delete;
    Staging& operator=(const Staging&) = delete;
};

