"""Template refinement by Adam on the template-projection loss, entirely on the device.

One step evaluates L(V) = P(V) + CD(mu(V), Y) (see autograd.py for the
definitions) and its gradient with the library's kernels, then applies Adam
(Kingma & Ba 2015, torch.optim.Adam's update):

  1. clear the gradient accumulators                     (mg_fill)
  2. refit the template BVH to V                          (mg_lbvh_refit)
  3. closest point on (V, F) of every target, starting
     from the previous step's face                        (mg_closest_point_query)
  4. P = mean squared distance                            (mg_mean)
  5. re-pose the Gaussian means mu(V)                     (mg_mesh_gaussian_update)
  6. refit the point LBVH over mu (built once from mu(V0):
     the means move little per step and nearest points stay
     exact on any tree), both nearest-neighbour maps from
     the previous step's, CD                              (mg_lbvh_refit, mg_chamfer)
  7. dP/dV, dCD/dmu, and dCD/dV through the binding       (mg_point_mesh_backward,
                                                           mg_chamfer_backward,
                                                           mg_mesh_gaussian_update_backward)
  8. Adam on V                                            (mg_adam_step)

No step synchronises with the host, so a whole run (reset + K steps) can be
captured in one HIP graph and replayed.  The loss of step s (at the V that
step starts from) is kept in history[s] = (P, CD a->b, CD b->a, L), float64.
"""

import math

import torch

from . import api


class TemplateRefiner:
    """Adam refinement of template vertices toward target samples.

    verts0 [3][V] float32, faces [3][F] int32, binding dict (face, bary,
    q_local, log_scale[, offset]) and targets [3][Y] float32, all on one
    device.  lr defaults to 1e-3 times the diagonal of verts0's bounding box.
    query / nn_query: traversal options for the closest-point and
    nearest-point queries.
    """

    def __init__(self, verts0, faces, binding, targets, *, lr=None, betas=(0.9, 0.999), eps=1e-8,
                 max_steps=200, query=None, nn_query=None):
        dev = verts0.device
        self.faces, self.binding, self.targets = faces, binding, targets
        self.verts0 = verts0
        self.frames0 = verts0.reshape(1, *verts0.shape)          # a one-frame store, copied by mg_vertex_buffer_update
        self.V = torch.empty_like(verts0)
        self.m = torch.empty_like(verts0)
        self.v = torch.empty_like(verts0)
        self.gV = torch.empty_like(verts0)
        G = binding["face"].shape[0]
        ny = targets.shape[1]
        self.G, self.ny = G, ny
        self.mu = torch.empty(3, G, device=dev)
        self.gmu = torch.empty(3, G, device=dev)
        self.rec = api._query_out(ny, dev, True, True, True, False)
        self.ch = {"nn_ab": torch.empty(G, dtype=torch.int32, device=dev), "d_ab": torch.empty(G, device=dev),
                   "nn_ba": torch.empty(ny, dtype=torch.int32, device=dev), "d_ba": torch.empty(ny, device=dev)}
        # each step's queries start from the previous step's answers (none at first)
        for t in (self.rec["face"], self.ch["nn_ab"], self.ch["nn_ba"]):
            t.fill_(-1)
        self.history = torch.zeros(max_steps, 4, dtype=torch.float64, device=dev)
        self.max_steps = max_steps
        self.bvh = api.lbvh_build(verts0, faces)
        self.bvh_y = api.lbvh_build(targets, None)
        mu0 = api.mesh_gaussian_update(verts0, faces, binding["face"], binding["bary"], binding["q_local"],
                                       binding["log_scale"], binding.get("offset"), quat=False, cov=False)["mean"]
        self.bvh_mu = api.lbvh_build(mu0, None)
        if lr is None:
            ext = (verts0.max(dim=1).values - verts0.min(dim=1).values).double()
            lr = 1e-3 * math.sqrt(float((ext * ext).sum()))
        self.lr, self.betas, self.eps = float(lr), betas, eps
        self.query = dict(query or {})
        self.nn_query = dict(nn_query or {})
        self.t = 0
        self.reset()

    def reset(self):
        """V <- verts0, Adam moments <- 0, step counter <- 0 (device work on the current stream)."""
        api.vertex_buffer_update(self.frames0, 0, self.V)
        api.fill(self.m, 0.0)
        api.fill(self.v, 0.0)
        self.t = 0

    def loss_and_grad(self, hist_row=None):
        """Evaluate L at the current V: fills gV (dL/dV) and, if given, a float64 [4] history row
        (P, CD a->b, CD b->a, L = P + CD, the last summed by mg_chamfer)."""
        b = self.binding
        api.fill(self.gV, 0.0)
        api.fill(self.gmu, 0.0)
        api.lbvh_refit(self.bvh, self.V)
        api.closest_point_query(self.bvh, self.V, self.targets, out=self.rec, hint=self.rec["face"], **self.query)
        row = hist_row if hist_row is not None else torch.empty(4, dtype=torch.float64, device=self.V.device)
        api.mean(self.rec["dist2"], out=row[0:1])
        api.mesh_gaussian_update(self.V, self.faces, b["face"], b["bary"], b["q_local"], b["log_scale"],
                                 b.get("offset"), out={"mean": self.mu}, quat=False, cov=False)
        api.lbvh_refit(self.bvh_mu, self.mu)
        api.chamfer(self.mu, self.bvh_mu, self.targets, self.bvh_y, out=dict(self.ch, loss=row[1:4]),
                    add=row[0:1], warm=True, **self.nn_query)
        if self.ny:
            api.point_mesh_backward(self.V, self.faces, self.targets, self.rec, 1.0 / self.ny, self.gV)
        if self.G:
            api.chamfer_backward(self.mu, self.targets, self.ch["nn_ab"], self.ch["nn_ba"], 1.0 / self.G,
                                 1.0 / self.ny if self.ny else 0.0, self.gmu)
            api.mesh_gaussian_update_backward(self.V, self.faces, b["face"], b["bary"], b["q_local"],
                                              b["log_scale"], b.get("offset"), self.gmu, g_verts=self.gV)
        return row

    def step(self):
        """One refinement step: loss and gradient at V into history[t], then Adam."""
        if self.t >= self.max_steps:
            raise ValueError(f"more than max_steps={self.max_steps} steps; reset() first")
        self.loss_and_grad(self.history[self.t])
        self.t += 1
        api.adam_step(self.V, self.gV, self.m, self.v, self.t, self.lr, self.betas[0], self.betas[1], self.eps)

    def run(self, steps):
        """reset() then `steps` steps (enqueued; nothing waits on the host)."""
        self.reset()
        for _ in range(steps):
            self.step()

    def capture(self, steps):
        """A torch.cuda.CUDAGraph of run(steps); replay() redoes the whole refinement from verts0."""
        self.run(1)                                   # warm every launch path before capture
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run(steps)
        return g

    def losses(self):
        """Host copy of the loss history so far: [t][4] (P, CD a->b, CD b->a, L)."""
        return self.history[:self.t].cpu()
