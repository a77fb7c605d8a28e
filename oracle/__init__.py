"""FP64 CPU oracle for graph-neural MPC linearization and condensing.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the test-suite, the smoke check and the CPU
baseline leg of the benchmark use it.  It shares no code with the HIP path;
both sides draw their inputs from ``paper_2602_17601_amd.workloads``.

Modules (each function cites the passage it follows):
  graph     -- neighbourhoods and the L-hop Jacobian pattern (Sec. III-A, Sec. V-B)
  msd       -- mass-spring-damper stand-in dynamics and analytic Jacobians
  gnn       -- the GNN dynamics model (Sec. V-A) and its per-node forward-mode
               linearization (Sec. V-A "Linearization", eq. linearized_dynamics)
  condense  -- dense condensing (Sec. III-B eq. condensed_matrices) and the
               paper's per-node recursion (Sec. V-B, Thm. 1 proof)
  qp        -- primal-dual interior-point QP solver and brute-force enumeration
  kkt       -- uncondensed equality-constrained KKT solve of the OCP (Sec. III-B eq. 2)
  tangent   -- products with the linearized model's blocks (forward and reverse mode)
  mpc       -- one iteration of the GNN-MPC loop with its shift (Algorithm 1)
  inet      -- the paper's own model, an interaction network with a global input
               (Sec. V-A eq. forward_dynamics), and its forward-mode linearization
  train     -- the training loss (weighted MSE plus an l2 penalty, Sec. V-A
               "Training"), its gradient by reverse mode, and the Adam update

Everything is float64.  Cost convention: stage cost 1/2 x'Qx + q'x + 1/2 u'Ru + r'u
and QP objective 1/2 u'Hu + g'u, under which the paper's formulas for H and g
hold exactly (the paper writes the norms without the factor 1/2 but its g has
no factor 2).
"""
