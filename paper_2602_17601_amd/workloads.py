"""Seeded synthetic workloads for graph-neural MPC on chain graphs.

This module only *constructs inputs*: graphs, model parameters, initial
states, nominal trajectories, cost weights and constraint rows.  It holds
none of the method's arithmetic (no dynamics, no Jacobians, no condensing),
so both the HIP path and the FP64 oracle can draw their inputs from it.

Every array is produced by ``numpy.random.default_rng(seed)`` (PCG64) in a
fixed draw order, in float64; callers cast to the precision they run in.

Readings of the paper that shape the inputs (Sec. IV-A, Sec. V-A):
  * the graph is a chain of M nodes with directed edges j -> i for
    1 <= |i - j| <= hops (both directions present, no self loops), stored as
    CSR indexed by the receiver i (the edge e^{ij} runs from v_j to v_i);
  * each node carries x^i = [p^i; v^i] in R^6; stacked states are node-major;
  * the inputs are 3D forces at a set of actuated nodes, u = [f_a1; f_a2; ...]
    in ascending node order, so n_u = 3 * n_act;
  * the synthetic nominal trajectory is a seeded random walk around x0 (the
    method linearizes around any given trajectory; it does not have to be a
    rollout of the model).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

NBX = 6  # states per node: position (3) and velocity (3)


# --------------------------------------------------------------------------
# graph
# --------------------------------------------------------------------------
def chain_csr(M: int, hops: int):
    """Incoming-edge CSR of a chain: row i lists j with 1 <= |i-j| <= hops."""
    row_ptr = np.zeros(M + 1, dtype=np.int32)
    cols = []
    for i in range(M):
        nb = [j for j in range(max(0, i - hops), min(M, i + hops + 1)) if j != i]
        cols.extend(nb)
        row_ptr[i + 1] = row_ptr[i] + len(nb)
    return row_ptr, np.asarray(cols, dtype=np.int32)


def actuated_nodes(M: int, n_act: int):
    """0-based actuated nodes: node ceil(a*M/n_act) (1-based) for a = 1..n_act.

    For M=10, n_act=2 this is nodes 5 and 10 (1-based); for n_act=4 it is
    M/4, M/2, 3M/4 and M.
    """
    return np.asarray([int(math.ceil(a * M / n_act)) - 1 for a in range(1, n_act + 1)],
                      dtype=np.int32)


# --------------------------------------------------------------------------
# model parameters
# --------------------------------------------------------------------------
@dataclass
class MSDParams:
    """Mass-spring-damper chain: springs/dampers along every graph edge."""
    k: float = 10.0
    c: float = 0.1
    m: float = 1.0
    dt: float = 0.01
    k3: float = 0.0          # cubic spring coefficient (0 = linear)
    gravity: float = 0.0     # magnitude of gravity along -z (0 = off)
    anchor: int = 0          # node tied to the ground by (k, c, k3)


@dataclass
class GNNWeights:
    """Weights of the message-passing GNN, float64, (out, in) row-major.

    enc: Hd x (6 + 3)   encoder on [x^i; P^i u]
    edge[l]: Hd x 2Hd   edge MLP on [h_i; h_i - h_j]
    node[l]: Hd x 2Hd   node MLP on [h_i; sum_j m_ij]
    dec: 6 x Hd         decoder; channels 3..5 are the velocity increment
    """
    Hd: int
    L: int
    W_enc: np.ndarray
    b_enc: np.ndarray
    W_edge: list
    b_edge: list
    W_node: list
    b_node: list
    W_dec: np.ndarray
    b_dec: np.ndarray
    dt: float = 0.01

    def rounded_bf16(self, biases: str = "bf16") -> "GNNWeights":
        """Copy with every weight rounded to bfloat16 (RNE), as float64; biases
        rounded to bfloat16 too (``biases='bf16'``) or to float32 (``'f32'``, how
        the library's BF16 mode holds them: added to FP32 sums)."""
        r = bf16_round
        rb = r if biases == "bf16" else (lambda b: np.asarray(b, np.float32).astype(np.float64))
        return GNNWeights(self.Hd, self.L, r(self.W_enc), rb(self.b_enc),
                          [r(w) for w in self.W_edge], [rb(b) for b in self.b_edge],
                          [r(w) for w in self.W_node], [rb(b) for b in self.b_node],
                          r(self.W_dec), rb(self.b_dec), self.dt)


@dataclass
class InetWeights:
    """The interaction network of Sec. V-A (eq. forward_dynamics), float64,
    (out, in) row-major: psi maps the relative state e^{ij} = x^i - x^j (6) to a
    message (d_m); phi maps [x^i (6); sum_j psi(e^{ij}) (d_m); u (n_u, the global
    input)] to the velocity increment (3).  Each is a list of linear layers with a
    ReLU after every layer but the last.  v+ = v + phi, p+ = p + dt v+."""
    psi_W: list
    psi_b: list
    phi_W: list
    phi_b: list
    nu: int
    dt: float = 0.01

    @property
    def d_m(self):
        return int(self.psi_W[-1].shape[0])

    def flat(self):
        """Weights packed as the library takes them: psi (W, b) per layer, then phi."""
        parts = []
        for W, b in list(zip(self.psi_W, self.psi_b)) + list(zip(self.phi_W, self.phi_b)):
            parts += [np.asarray(W, np.float64).reshape(-1), np.asarray(b, np.float64).reshape(-1)]
        return np.concatenate(parts)


def inet_weights(seed: int, nu: int = 6, psi_hidden: int = 4, psi_width: int = 50, d_m: int = 50,
                 phi_hidden: int = 8, phi_width: int = 250, dt: float = 0.01, bias_lo: float = -0.1,
                 bias_hi: float = 0.1) -> InetWeights:
    """Xavier-uniform weights (gain 1) for psi then phi, layer by layer; biases
    uniform in [bias_lo, bias_hi) drawn after all weights (a range above zero
    makes every ReLU active for inputs near zero)."""
    rng = np.random.default_rng(seed)
    psi_dims = [6] + [psi_width] * psi_hidden + [d_m]
    phi_dims = [6 + d_m + nu] + [phi_width] * phi_hidden + [3]
    psi_W = [xavier(rng, psi_dims[l + 1], psi_dims[l]) for l in range(len(psi_dims) - 1)]
    phi_W = [xavier(rng, phi_dims[l + 1], phi_dims[l]) for l in range(len(phi_dims) - 1)]
    psi_b = [rng.uniform(bias_lo, bias_hi, psi_dims[l + 1]) for l in range(len(psi_dims) - 1)]
    phi_b = [rng.uniform(bias_lo, bias_hi, phi_dims[l + 1]) for l in range(len(phi_dims) - 1)]
    return InetWeights(psi_W, psi_b, phi_W, phi_b, nu, dt)


def nearest_csr(M: int, d: int):
    """Incoming-edge CSR where node i's senders are the d other nodes nearest to it
    in index (ties toward the lower index), rows ascending."""
    row_ptr, col = [0], []
    for i in range(M):
        others = sorted((j for j in range(M) if j != i), key=lambda j: (abs(j - i), j))[:d]
        col += sorted(others)
        row_ptr.append(len(col))
    return np.asarray(row_ptr, np.int32), np.asarray(col, np.int32)


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round float64 values to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def xavier(rng, fan_out: int, fan_in: int):
    bound = math.sqrt(6.0 / (fan_in + fan_out))
    return rng.uniform(-bound, bound, size=(fan_out, fan_in))


def gnn_weights(seed: int, Hd: int, L: int, dt: float = 0.01, nin: int = 9,
                nout: int = 6, bias_scale: float = 0.0) -> GNNWeights:
    """Xavier-uniform weights (gain 1), drawn enc, (edge, node) x L, dec.

    Biases are zero unless ``bias_scale`` > 0, in which case they are drawn
    uniformly from [0, bias_scale) after all weights (used by tests that need
    every ReLU active).
    """
    rng = np.random.default_rng(seed)
    W_enc = xavier(rng, Hd, nin)
    W_edge, W_node = [], []
    for _ in range(L):
        W_edge.append(xavier(rng, Hd, 2 * Hd))
        W_node.append(xavier(rng, Hd, 2 * Hd))
    W_dec = xavier(rng, nout, Hd)
    if bias_scale > 0:
        b_enc = rng.uniform(0, bias_scale, Hd)
        b_edge = [rng.uniform(0, bias_scale, Hd) for _ in range(L)]
        b_node = [rng.uniform(0, bias_scale, Hd) for _ in range(L)]
        b_dec = rng.uniform(0, bias_scale, nout)
    else:
        b_enc = np.zeros(Hd)
        b_edge = [np.zeros(Hd) for _ in range(L)]
        b_node = [np.zeros(Hd) for _ in range(L)]
        b_dec = np.zeros(nout)
    return GNNWeights(Hd, L, W_enc, b_enc, W_edge, b_edge, W_node, b_node, W_dec, b_dec, dt)


# --------------------------------------------------------------------------
# trajectories, costs, constraints
# --------------------------------------------------------------------------
def initial_state(rng, M: int, sigma: float):
    return rng.normal(0.0, sigma, size=(M, NBX))


def nominal_trajectory(rng, x0, N: int, nu: int, walk: float):
    """x_hat[0] = x0, x_hat[k+1] = x_hat[k] + walk * N(0, 1); u_hat ~ U(-1, 1)."""
    M = x0.shape[0]
    xhat = np.empty((N + 1, M, NBX))
    xhat[0] = x0
    for k in range(N):
        xhat[k + 1] = xhat[k] + walk * rng.normal(size=(M, NBX))
    uhat = rng.uniform(-1.0, 1.0, size=(N, nu))
    return xhat, uhat


@dataclass
class Costs:
    Q: np.ndarray      # [N+1][M][6] diagonal, or [N+1][M][6][6] full
    q: np.ndarray      # [N+1][M][6]
    R: np.ndarray      # [N][nu][nu]
    r: np.ndarray      # [N][nu]
    full_Q: bool = False


def tracking_costs(M: int, N: int, nu: int, qdiag, rho_r: float):
    Q = np.broadcast_to(np.asarray(qdiag, dtype=np.float64), (N + 1, M, NBX)).copy()
    R = np.broadcast_to(rho_r * np.eye(nu), (N, nu, nu)).copy()
    return Costs(Q, np.zeros((N + 1, M, NBX)), R, np.zeros((N, nu)))


def random_costs(rng, M: int, N: int, nu: int, full_Q: bool = False):
    """Random positive-definite stage costs with nonzero linear terms."""
    if full_Q:
        G = rng.normal(size=(N + 1, M, NBX, NBX))
        Q = np.einsum("kmab,kmcb->kmac", G, G) / NBX + 0.1 * np.eye(NBX)
    else:
        Q = rng.uniform(0.1, 2.0, size=(N + 1, M, NBX))
    G = rng.normal(size=(N, nu, nu))
    R = np.einsum("kab,kcb->kac", G, G) / nu + 0.1 * np.eye(nu)
    q = rng.normal(size=(N + 1, M, NBX))
    r = rng.normal(size=(N, nu))
    return Costs(Q, q, R, r, full_Q)


@dataclass
class StateRows:
    """Half-space rows C x^i_k <= d on single nodes (Sec. IV-B)."""
    node: np.ndarray    # int32 [n_c]
    stage: np.ndarray   # int32 [n_c], 1..N
    C: np.ndarray       # [n_c][6]
    d: np.ndarray       # [n_c]

    @property
    def n(self):
        return int(self.node.shape[0])


def no_rows():
    return StateRows(np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros((0, NBX)), np.zeros(0))


def random_rows(rng, M: int, N: int, n_c: int):
    node = rng.integers(0, M, size=n_c).astype(np.int32)
    stage = rng.integers(1, N + 1, size=n_c).astype(np.int32)
    C = rng.normal(size=(n_c, NBX))
    d = rng.normal(size=n_c)
    return StateRows(node, stage, C, d)


def sphere_obstacle_rows(rng, M: int, N: int, xhat, act, radius: float = 0.1,
                         clearance: float = 0.15, n_nodes: int = 10, spread: int = 8):
    """Node-position half-spaces keeping nodes outside a sphere obstacle.

    Rest positions hang along -z: r^i = (0, 0, -i/M).  The sphere (radius
    ``radius``) sits beside a seeded node c at distance ``clearance`` along a
    seeded horizontal unit vector; c is drawn within ``spread`` nodes of the
    actuated node nearest the middle of the chain, so that the inputs reach
    the constrained nodes within the horizon (a row no input reaches has
    C S_k = 0 and only restates a fact about the free response).  For each of the
    ``n_nodes`` nodes nearest the centre and each stage k = 1..N, the row
    linearizes "outside the sphere" around the nominal position:
    n = unit(r^i + p_hat^i_k - centre), C = [-n^T, 0], d = n^T (r^i - centre) - radius,
    so that C x^i_k <= d  <=>  n^T (r^i + p^i_k - centre) >= radius.
    """
    rest = np.zeros((M, 3))
    rest[:, 2] = -np.arange(M) / M
    a_mid = int(np.asarray(act)[np.argmin(np.abs(np.asarray(act) - (M - 1) / 2))])
    c = min(M - 1, max(0, a_mid + int(rng.integers(-spread, spread + 1))))
    ang = rng.uniform(0, 2 * math.pi)
    w = np.array([math.cos(ang), math.sin(ang), 0.0])
    centre = rest[c] + clearance * w
    dist = np.linalg.norm(rest - centre, axis=1)
    nodes = np.sort(np.argsort(dist, kind="stable")[:n_nodes])
    node, stage, C, d = [], [], [], []
    for k in range(1, N + 1):
        for i in nodes:
            v = rest[i] + xhat[k, i, :3] - centre
            n = v / np.linalg.norm(v)
            node.append(i)
            stage.append(k)
            C.append(np.concatenate([-n, np.zeros(3)]))
            d.append(float(n @ (rest[i] - centre)) - radius)
    return StateRows(np.asarray(node, np.int32), np.asarray(stage, np.int32),
                     np.asarray(C), np.asarray(d))


# --------------------------------------------------------------------------
# complete problem instances
# --------------------------------------------------------------------------
@dataclass
class Problem:
    name: str
    M: int
    hops: int
    N: int
    act: np.ndarray
    row_ptr: np.ndarray
    col: np.ndarray
    x0: np.ndarray
    xhat: np.ndarray
    uhat: np.ndarray
    costs: Costs
    rows: StateRows
    lb: np.ndarray
    ub: np.ndarray
    model: str                      # "msd", "gnn" or "inet"
    msd: MSDParams = field(default_factory=MSDParams)
    gnn: GNNWeights | None = None
    dtype: str = "f32"              # arithmetic of condensing: "f64" | "f32"
    gnn_dtype: str = "f32"          # arithmetic of the GNN MLPs: "f32" | "bf16"
    inet: InetWeights | None = None

    @property
    def nu(self):
        return self.inet.nu if self.model == "inet" else 3 * len(self.act)

    @property
    def L(self):
        return self.gnn.L if self.model == "gnn" else 1

    @property
    def E(self):
        return int(self.col.shape[0])


def make_problem(name: str, *, M: int, hops: int, N: int, n_act: int, model: str,
                 seed: int, Hd: int = 64, L: int = 2, weight_seed: int | None = None,
                 x0_sigma: float = 0.1, walk: float = 0.0, qdiag=(1, 1, 1, .01, .01, .01),
                 rho_r: float = 0.1, obstacle: bool = False, random_cost: bool = False,
                 full_Q: bool = False, n_random_rows: int = 0, umax: float = 1.0,
                 msd: MSDParams | None = None, dtype: str = "f32", gnn_dtype: str = "f32",
                 bias_scale: float = 0.0) -> Problem:
    """Build one seeded instance.  Draw order: weights (own seed), x0, x_hat/u_hat,
    then obstacle or random rows, then random costs."""
    act = actuated_nodes(M, n_act)
    nu = 3 * n_act
    row_ptr, col = chain_csr(M, hops)
    gnn = None
    if model == "gnn":
        gnn = gnn_weights(seed if weight_seed is None else weight_seed, Hd, L,
                          dt=(msd or MSDParams()).dt, bias_scale=bias_scale)
    rng = np.random.default_rng(seed)
    x0 = initial_state(rng, M, x0_sigma)
    xhat, uhat = nominal_trajectory(rng, x0, N, nu, walk)
    if obstacle:
        rows = sphere_obstacle_rows(rng, M, N, xhat, act)
    elif n_random_rows:
        rows = random_rows(rng, M, N, n_random_rows)
    else:
        rows = no_rows()
    if random_cost:
        costs = random_costs(rng, M, N, nu, full_Q)
    else:
        costs = tracking_costs(M, N, nu, qdiag, rho_r)
    lb = -umax * np.ones(N * nu)
    ub = umax * np.ones(N * nu)
    return Problem(name, M, hops, N, act, row_ptr, col, x0, xhat, uhat, costs, rows, lb, ub,
                   model, msd or MSDParams(), gnn, dtype, gnn_dtype)


def msd10_fp64() -> Problem:
    """Plain condensing in FP64: linear MSD chain of 10 nodes, nearest-neighbour
    edges, forces at nodes 5 and 10, N=10, Q=I, R=0.1I, |u|<=1, x0 ~ N(0, 0.1^2)."""
    return make_problem("msd10_fp64", M=10, hops=1, N=10, n_act=2, model="msd", seed=0,
                        x0_sigma=0.1, qdiag=(1, 1, 1, 1, 1, 1), dtype="f64")


def gnn100_fp32(model: str = "gnn") -> Problem:
    """GNN-linearized condensing in FP32: 100-node 1-2-hop chain, Hd=64, L=2,
    forces at nodes 50 and 100, N=20.  ``model='msd'`` gives the plain form."""
    return make_problem("gnn100_fp32" if model == "gnn" else "msd100_fp32", M=100, hops=2, N=20, n_act=2,
                        model=model, seed=2, weight_seed=1, Hd=64, L=2, x0_sigma=0.02, walk=0.002)


def gnn1000_bf16(model: str = "gnn") -> Problem:
    """Paper-scale single instance: 1000-node 1-2-hop chain, Hd=128, L=3 (BF16
    MLPs, FP32 condensing), forces at 4 nodes (n_u=12), N=20, 200 obstacle rows.
    ``model='msd'`` gives the plain (analytic-Jacobian) form on the same graph."""
    return make_problem("gnn1000_bf16" if model == "gnn" else "msd1000_fp32",
                        M=1000, hops=2, N=20, n_act=4, model=model, seed=3, Hd=128, L=3,
                        x0_sigma=0.02, walk=0.002, obstacle=True,
                        gnn_dtype="bf16" if model == "gnn" else "f32")


def trunk_inet(M: int = 4, d: int = 2, N: int = 20, nu: int = 6, seed: int = 7, x0_sigma: float = 0.02,
               walk: float = 0.002, umax: float = 1.0, **inet_kw) -> Problem:
    """The paper's own model on its robot's shape (Sec. VI-C): M = 4 nodes with d = 2
    neighbours each, the interaction network with psi 4 x 50 and phi 8 x 250 hidden
    units and a global input of n_u = 6 (six motors), N = 20 at 100 Hz; seeded
    random weights (no trained ones exist here), tracking costs, |u| <= umax."""
    row_ptr, col = nearest_csr(M, d)
    W = inet_weights(seed, nu=nu, **inet_kw)
    rng = np.random.default_rng(seed + 1)
    x0 = initial_state(rng, M, x0_sigma)
    xhat, uhat = nominal_trajectory(rng, x0, N, nu, walk)
    costs = tracking_costs(M, N, nu, (1, 1, 1, .01, .01, .01), 0.1)
    return Problem(f"trunk_inet{M}", M, 0, N, np.zeros(0, np.int32), row_ptr, col, x0, xhat, uhat, costs, no_rows(),
                   -umax * np.ones(N * nu), umax * np.ones(N * nu), "inet", MSDParams(dt=W.dt), None, "f32", "f32", W)


def batch_instances(count: int, seed: int = 4, M_range=(50, 1000), N_range=(10, 30)) -> list[Problem]:
    """A batch of independent instances of uneven size (the serving shape):
    instance i draws M ~ U{M_range}, N ~ U{N_range} and 2, 3 or 4 actuated nodes
    from ``default_rng(seed)``; all share one GNN (Hd=128, L=2, BF16 MLPs, FP32
    condensing, weights from ``seed``), tracking costs, |u| <= 1 and no state rows."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        M = int(rng.integers(M_range[0], M_range[1] + 1))
        N = int(rng.integers(N_range[0], N_range[1] + 1))
        n_act = int(rng.integers(2, 5))
        out.append(make_problem(f"batch{seed}_{i}", M=M, hops=2, N=N, n_act=n_act, model="gnn",
                                seed=seed * 100003 + i, weight_seed=seed, Hd=128, L=2, x0_sigma=0.02,
                                walk=0.002, gnn_dtype="bf16"))
    return out


@dataclass
class SimBatch:
    """Inputs of a batch of simulator trajectories on one chain."""
    name: str
    M: int
    hops: int
    act: np.ndarray
    row_ptr: np.ndarray
    col: np.ndarray
    msd: MSDParams
    x0: np.ndarray      # [B][M][6]
    u: np.ndarray       # [B][T][nu]

    @property
    def nu(self):
        return 3 * len(self.act)


def simulator_batch(B: int, T: int, M: int = 1000, hops: int = 2, n_act: int = 4, seed: int = 5,
                    x0_sigma: float = 0.02, step: float = 0.1) -> SimBatch:
    """Trajectory inputs for the learned-surrogate data set: the nonlinear chain
    (cubic springs k3 = 50, gravity 9.81, node 0 anchored), x0 ~ N(0, x0_sigma^2)
    per entry, and inputs as random walks u_0 ~ U(-1, 1), u_{t+1} = clip(u_t +
    step N(0, 1), -1, 1), all from ``default_rng(seed)`` (x0 first, then u)."""
    rng = np.random.default_rng(seed)
    act = actuated_nodes(M, n_act)
    row_ptr, col = chain_csr(M, hops)
    nu = 3 * n_act
    x0 = rng.normal(0.0, x0_sigma, size=(B, M, NBX))
    u = np.empty((B, T, nu))
    cur = rng.uniform(-1.0, 1.0, size=(B, nu))
    for t in range(T):
        u[:, t] = cur
        cur = np.clip(cur + step * rng.normal(size=(B, nu)), -1.0, 1.0)
    return SimBatch(f"sim{seed}_{B}x{T}x{M}", M, hops, act, row_ptr, col,
                    MSDParams(k3=50.0, gravity=9.81), x0, u)

