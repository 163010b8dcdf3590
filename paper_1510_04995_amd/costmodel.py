"""Learned cost model for the auto-tuner.

The paper's auto-tuner (Section "Auto-tuning") measures candidates: per
thread-group shape it hill-climbs over the diamond width, or it tries every
feasible point.  This module adds a learned proposer beside it.  A small
fully connected network predicts the log throughput of a candidate from its
features.  It is trained on the tuner's own measurements, and it proposes the
top-k candidates of a new problem.  The tuner then measures only those
(``GIRIH_TUNE_MODEL``).  Exhaustive search stays as the fallback and as the
reference the proposals are checked against.

All arithmetic of the network (forward, back-propagation, Adam) runs in the
``girih_mlp_*`` HIP kernels of ``libgirih.so``; this module holds the
features, the parameter initialisation and the training loop, with PyTorch
providing device memory and the stream.

Features of a candidate (22, in this order):
  0 stencil radius R          1 number of coefficient arrays
  2-4 log2 nx, ny, nz          5 dtype (0 = FP64, 1 = FP32)
  6 diamond width Dw           7 wavefront depth N_F
  8 log2 x tile                9 y tile (= Dw)
  10 log2 z tile               11 threads along x / 64 (waves along x)
  12 threads along y (row pairs)  13 x cells per lane
  14 LDS bytes / 64 KiB        15 log2 T
  16 schedule (variant bit 0: dependency-driven)
  17 synchronisation (variant bit 1: relaxed)
  18 log2 of the paper's blocked code balance B_C (bytes per update,
     Section "Memory traffic model"; N_D = 2 + coefficient arrays)
  19 log2 of the redundant x-halo read factor (x tile + 2R(L-1)) / x tile
  20 log2 of the rounds a diamond row's workgroups take on the 256 CUs
     (x chunks x diamonds of the row, over the CUs times the workgroups one
     CU holds by its LDS)
  21 fill of those rounds (workgroups / (rounds x slots))
They are standardised with the mean and spread of the training set.
Features 18 and 19 carry the traffic model across stencils: a problem whose
coefficient arrays the training set never saw still differs from the
training problems in B_C, which the training set relates to throughput.
The last two carry launch quantisation across grids: a tile that fits a
row's workgroups in one round on one grid can need two on another.
"""
import math

import numpy as np

from . import girih as G

N_FEATURES = 22
N_CU = 256
LDS_PER_CU = 163840
STENCIL_NCOEF = G.N_COEF
RADIUS = G.RADIUS


def features(stencil, dtype, nx, ny, nz, T, params, lds_bytes):
    """The 22 raw features of one candidate (see the module docstring)."""
    q = params
    v = int(q.get("variant") or 0)
    R, dw, tx = RADIUS[stencil], float(q["diamond_width"]), float(max(1, q["tile_x"]))
    s = 8.0 if dtype == "f64" else 4.0
    nd = 2 + STENCIL_NCOEF[stencil]
    b_c = 2 * s * R * ((2 * dw - 2 * R) + (nd * dw + 2 * R)) / (dw * dw)
    rho = (tx + 2 * R * (dw / R - 1)) / tx
    idw = int(q["diamond_width"])
    tiles = -(-nx // max(1, int(q["tile_x"]))) * ((ny + idw // 2 + idw - 1) // idw)
    slots = N_CU * max(1, LDS_PER_CU // max(1, int(lds_bytes)))
    rounds = -(-tiles // slots)
    return [float(RADIUS[stencil]), float(STENCIL_NCOEF[stencil]), math.log2(nx), math.log2(ny), math.log2(nz),
            0.0 if dtype == "f64" else 1.0, float(q["diamond_width"]), float(q["wavefront_depth"] or 1),
            math.log2(max(1, q["tile_x"])), float(q["tile_y"]), math.log2(max(1, q["tile_z"])),
            q["threads_x"] / 64.0, float(q["threads_y"]), float(q.get("cells_per_lane") or 1),
            lds_bytes / 65536.0, math.log2(max(1, T)), float(v & 1), float((v >> 1) & 1), math.log2(b_c),
            math.log2(rho), math.log2(rounds), tiles / (rounds * slots)]


def candidate_table(sweep, T):
    """[(params, raw features)] of every feasible MWD candidate of a plan.

    LDS bytes come from the plan itself (plan_info after set_params, host
    only); the plan's own parameters are restored afterwards."""
    saved = sweep.info()["params"]
    out = []
    try:
        for q in sweep.candidates():
            sweep.set_params(q)
            info = sweep.info()
            out.append((info["params"], features(sweep.stencil, sweep.dtype, sweep.nx, sweep.ny, sweep.nz, T,
                                                 info["params"], info["lds_bytes"])))
    finally:
        sweep.set_params(saved)
    return out


def records_from_log(sweep, T, log):
    """(raw features, GLUP/s) of every successfully measured tuner record."""
    X, y = [], []
    for r in log:
        if r["status"] != 0 or not (r["glups"] > 0):
            continue
        X.append(features(sweep.stencil, sweep.dtype, sweep.nx, sweep.ny, sweep.nz, T, r["params"], r["lds_bytes"]))
        y.append(r["glups"])
    return X, y


def he_uniform(n_in, n_hidden, n_layers, seed=0):
    """Initial parameters (flat, FP32): He-uniform weights, zero biases, drawn
    from numpy's PCG64 generator in layer order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shapes = [(n_hidden, n_in)] + [(n_hidden, n_hidden)] * (n_layers - 1) + [(1, n_hidden)]
    parts = []
    for fo, fi in shapes:
        lim = math.sqrt(6.0 / fi)
        parts.append(rng.uniform(-lim, lim, fo * fi))
        parts.append(np.zeros(fo))
    return np.concatenate(parts).astype(np.float32)


class CostModel:
    """A 20 -> n_layers x n_hidden (ReLU) -> 1 network predicting log GLUP/s."""

    def __init__(self, n_hidden=64, n_layers=3, seed=0, device=None):
        import torch
        self.torch = torch
        self.dev = device or torch.device("cuda:0")
        self.n_in, self.n_hidden, self.n_layers = N_FEATURES, n_hidden, n_layers
        self.count = G.girih_mlp_param_count(self.n_in, n_hidden, n_layers)
        p0 = he_uniform(self.n_in, n_hidden, n_layers, seed)
        assert p0.size == self.count
        self.params = torch.from_numpy(p0).to(self.dev)
        self.mean = np.zeros(self.n_in)
        self.scale = np.ones(self.n_in)

    def _norm(self, X):
        X = np.asarray(X, dtype=np.float64)
        return ((X - self.mean) / self.scale).astype(np.float32)

    def fit(self, X, glups, steps=3000, lr=3e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        """Full-batch Adam on the mean squared error of log GLUP/s; returns the
        loss after every step (a host copy, read at the end)."""
        torch = self.torch
        X = np.asarray(X, dtype=np.float64)
        self.mean = X.mean(axis=0)
        sd = X.std(axis=0)
        # a feature with no spread in the training set carries no information
        # the network could have learned: it standardises to 0 for every
        # candidate (e.g. the number of coefficient arrays when training saw
        # constant-coefficient stencils only)
        self.scale = np.where(sd > 1e-12, sd, np.inf)
        x = torch.from_numpy(self._norm(X)).to(self.dev).contiguous()
        t = torch.from_numpy(np.log(np.asarray(glups, dtype=np.float64)).astype(np.float32)).to(self.dev)
        n = x.shape[0]
        work_len = G.girih_mlp_work_count(self.n_in, self.n_hidden, self.n_layers, n)
        work = torch.empty(work_len, dtype=torch.float32, device=self.dev)
        grad = torch.empty(self.count, dtype=torch.float32, device=self.dev)
        m = torch.zeros(self.count, dtype=torch.float32, device=self.dev)
        v = torch.zeros(self.count, dtype=torch.float32, device=self.dev)
        losses = torch.empty(steps, dtype=torch.float32, device=self.dev)
        s = torch.cuda.current_stream().cuda_stream
        for k in range(steps):
            G.girih_mlp_loss_grad(self.params.data_ptr(), self.n_in, self.n_hidden, self.n_layers, x.data_ptr(),
                                  t.data_ptr(), n, losses[k:k + 1].data_ptr(), grad.data_ptr(), work.data_ptr(),
                                  work_len, s)
            G.girih_mlp_adam(self.params.data_ptr(), grad.data_ptr(), m.data_ptr(), v.data_ptr(), self.count, lr,
                             beta1, beta2, eps, k + 1, s)
        return losses.cpu().numpy()

    def predict(self, X):
        """Predicted GLUP/s of each row of raw features."""
        torch = self.torch
        x = torch.from_numpy(self._norm(X)).to(self.dev).contiguous()
        n = x.shape[0]
        work_len = G.girih_mlp_work_count(self.n_in, self.n_hidden, self.n_layers, n)
        work = torch.empty(work_len, dtype=torch.float32, device=self.dev)
        y = torch.empty(n, dtype=torch.float32, device=self.dev)
        G.girih_mlp_forward(self.params.data_ptr(), self.n_in, self.n_hidden, self.n_layers, x.data_ptr(), n,
                            y.data_ptr(), work.data_ptr(), work_len, torch.cuda.current_stream().cuda_stream)
        return np.exp(y.cpu().numpy().astype(np.float64))

    def propose(self, sweep, T, k=5):
        """k candidates of a plan to measure.  Candidates are grouped by
        workgroup shape (diamond width, waves along x, cells per lane) and
        the shapes ranked by their best prediction; the k picks go round
        robin over the shapes in that order, each shape's candidates in
        predicted order: the best candidate of each of the k leading
        shapes, or, where a problem has fewer shapes, their second-best
        next.  The paper's tuner searches each thread-group shape on its
        own; a model error about which shape is fastest -- the likeliest
        error on a problem unlike the training problems -- then cannot take
        all k measurements."""
        table = candidate_table(sweep, T)
        if not table:
            return []
        pred = self.predict([f for _, f in table])
        groups = {}
        for i in np.argsort(-pred, kind="stable"):
            q = table[i][0]
            groups.setdefault((q["diamond_width"], q["threads_x"], q["cells_per_lane"]), []).append(int(i))
        ranked = sorted(groups.values(), key=lambda g: -pred[g[0]])
        picks = []
        for r in range(k):
            for g in ranked:
                if r < len(g) and len(picks) < k:
                    picks.append(g[r])
        return [table[i][0] for i in picks]


def tune_with_model(sweep, model, T, k=5, max_seconds=60.0):
    """Measure only the model's top-k candidates; returns (best params, GLUP/s,
    number of candidates measured)."""
    cands = model.propose(sweep, T, k)
    sweep.set_candidates(cands)
    n_before = len(sweep.tune_log())
    best, rate = sweep.tune("model", T, max_seconds)
    return best, rate, len(sweep.tune_log()) - n_before


def retime(sweep, T, picks, rounds=3, max_seconds=60.0):
    """Time the given parameter sets together, interleaved over `rounds`
    rounds with the tuner's own measurement: {index: median GLUP/s}.  Used to
    compare the picks of different searches under the same conditions (a
    search's own best figure carries the noise of the moment it was taken)."""
    cands = [picks[i] for _ in range(rounds) for i in range(len(picks))]
    sweep.set_candidates(cands)
    n0 = len(sweep.tune_log())
    sweep.tune("model", T, max_seconds)
    log = sweep.tune_log()[n0:]
    out = {}
    for i, p in enumerate(picks):
        vals = sorted(r["glups"] for j, r in enumerate(log) if j % len(picks) == i and r["status"] == 0)
        out[i] = vals[len(vals) // 2] if vals else 0.0
    return out

