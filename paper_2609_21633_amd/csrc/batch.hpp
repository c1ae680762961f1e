// Lockstep batch of Stokes solver slots on one mesh (serving): every kernel of
// an FGMRES iteration runs once for all running slots (grid x slots), each
// slot with its own viscosity, right-hand side, eigenvalue estimates, Krylov
// basis and convergence test.
#pragma once

#include <chrono>
#include <memory>
#include <vector>

#include "tng_internal.hpp"

namespace tng {

// Solver as tng_stokes_solver_create builds it; batch_slot adds the buffers a
// batch slot needs (index-free preconditioner output).
tng_solver* create_solver(tng_ctx* ctx, tng_mesh* mesh, const tng_solver_opts* opts, bool batch_slot);

class SolverBatch {
  public:
    // Slots solve in ctx's stream; opts as for a single solver (mixed or FP64).
    SolverBatch(tng_ctx* ctx, tng_mesh* mesh, const tng_solver_opts& opts);
    ~SolverBatch();
    SolverBatch(const SolverBatch&) = delete;
    SolverBatch& operator=(const SolverBatch&) = delete;

    // Device bytes of one slot (its arena), measured by building one slot.
    long long slot_bytes() const { return slot_bytes_; }
    int slots() const { return (int)slot_.size(); }
    int running() const;
    // Index of an idle slot, or -1.
    int idle_slot() const;
    // Adds an idle slot (one arena allocation); returns its index.
    int add_slot();
    // Frees idle slot i; later slots move down by one index.
    void remove_slot(int i);

    // Slot i takes the problem eta = exp(-E T), f = Ra T rhat, g = 0 (T: nodal
    // FP64 field of the mesh's level 0); set-up runs now.  The result goes to
    // u_out, p_out when the slot finishes.  Returns false if the problem
    // failed in set-up (the slot is idle again; see result()).
    bool start(int i, const double* T, double E, double Ra, double* const u_out[3], double* p_out);
    // One FGMRES iteration of every running slot, then the restart and
    // refinement work of the slots whose Krylov cycle ended; returns the
    // slots that finished in this step (their results are written).
    std::vector<int> step();
    // Outcome of the last problem of slot i.
    int rc(int i) const;
    tng_solve_info info(int i) const;

    struct Slot;
    struct Staging;

  private:
    tng_ctx* ctx_;
    tng_mesh* mesh_;
    tng_solver_opts opts_;
    long long slot_bytes_ = 0;
    std::vector<std::unique_ptr<Slot>> slot_;
    std::unique_ptr<Staging> st_;
};

}  // namespace tng
