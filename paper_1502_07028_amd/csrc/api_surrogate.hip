// C ABI of the learned first stage of delayed acceptance (declared in
// include/tca.h): surrogate objects, dataset collection from exact sweeps,
// training, evaluation and attachment to a lattice context.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <vector>

#include "ctx.hpp"
#include "surrogate.hpp"

using namespace tca;

namespace {

constexpr int kEvalChunk = 4096;  // rows per evaluation launch

bool valid_hidden(int H) { return H >= 16 && H <= 1024 && H % 16 == 0; }

// Training buffers for `rows` rows (grow only).
hipError_t ensure_train_bufs(tca_surrogate* s, int rows) {
  if (rows <= s->tb_rows) return hipSuccess;
  const size_t H = s->dm.hidden, nin = s->dm.n_in, r = rows;
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = s->Xb.alloc(r * nin);
  if (e == hipSuccess) e = s->yb.alloc(r);
  if (e == hipSuccess) e = s->z1.alloc(r * H);
  if (e == hipSuccess) e = s->h1.alloc(r * H);
  if (e == hipSuccess) e = s->z2.alloc(r * H);
  if (e == hipSuccess) e = s->h2.alloc(r * H);
  if (e == hipSuccess) e = s->out.alloc(r);
  if (e == hipSuccess) e = s->dout.alloc(r);
  if (e == hipSuccess) e = s->dz1.alloc(r * H);
  if (e == hipSuccess) e = s->dz2.alloc(r * H);
  if (e == hipSuccess) e = s->dh.alloc(r * H);
  s->tb_rows = e == hipSuccess ? rows : 0;
  return e;
}

SgTrainBufs train_bufs(tca_surrogate* s, double* loss) {
  return SgTrainBufs{s->Xb.p, s->yb.p, s->z1.p, s->h1.p, s->z2.p, s->h2.p, s->out.p,
                     s->dz1.p, s->dz2.p, s->dh.p, s->dout.p, loss};
}

// Sum of squared errors of the FP32 (bf16 = false) or BF16 network over
// dataset rows [r0, r1).
int holdout_sse(tca_surrogate* s, int64_t r0, int64_t r1, bool bf16, double* sse) {
  *sse = 0.0;
  if (r1 <= r0) return TCA_OK;
  if (ensure_train_bufs(s, kEvalChunk) != hipSuccess) {
    set_err("training buffer allocation failed");
    return TCA_E_NOMEM;
  }
  const int H = s->dm.hidden;
  DevBuf<uint16_t> Fb, H1, H2;
  DevBuf<double> part;
  if (bf16) {
    TCA_CK(Fb.alloc((size_t)kEvalChunk * s->dm.kpad));
    TCA_CK(H1.alloc((size_t)kEvalChunk * H));
    TCA_CK(H2.alloc((size_t)kEvalChunk * H));
    if (s->bf16_stale) {
      TCA_CK(sg_to_bf16(s->W.p, s->dm, s->W1b.p, s->W2b.p, s->stream));
      s->bf16_stale = false;
    }
  }
  const int64_t nchunk = (r1 - r0 + kEvalChunk - 1) / kEvalChunk;
  TCA_CK(part.alloc((size_t)nchunk));
  for (int64_t ck = 0; ck < nchunk; ++ck) {
    const int64_t a = r0 + ck * kEvalChunk;
    const int rows = (int)((r1 - a) < kEvalChunk ? (r1 - a) : kEvalChunk);
    const float* X = s->X.p + a * s->dm.n_in;
    if (bf16) {
      TCA_CK(sg_f32_to_bf16_rows(X, rows, s->dm.n_in, s->dm.kpad, Fb.p, s->stream));
      TCA_CK(sg_infer_bf16(Fb.p, rows, s->W.p, s->W1b.p, s->W2b.p, s->dm,
                           SgInferBufs{H1.p, H2.p}, s->out.p, s->stream));
    } else {
      SgTrainBufs b = train_bufs(s, nullptr);
      TCA_CK(hipMemcpyAsync(b.Xb, X, sizeof(float) * rows * s->dm.n_in,
                            hipMemcpyDeviceToDevice, s->stream));
      TCA_CK(sg_forward(s->W.p, s->dm, rows, b, s->stream));
    }
    TCA_CK(sg_sse(s->out.p, s->y.p + a, rows, part.p + ck, s->stream));
  }
  std::vector<double> h(nchunk);
  TCA_CK(hipMemcpyAsync(h.data(), part.p, sizeof(double) * nchunk, hipMemcpyDeviceToHost,
                        s->stream));
  TCA_CK(hipStreamSynchronize(s->stream));
  for (double v : h) *sse += v;
  return TCA_OK;
}

}  // namespace

extern "C" {

int tca_surrogate_create(int32_t Lc, int32_t hidden, uint64_t seed, int64_t capacity,
                         void* hip_stream, tca_surrogate** out) {
  g_err[0] = 0;
  if (!out) TCA_INVAL("out is NULL");
  *out = nullptr;
  if (Lc < 2 || Lc > kMaxLc) TCA_INVAL("Lc must be 2..10");
  if (!valid_hidden(hidden)) TCA_INVAL("hidden must be 16..1024 and a multiple of 16");
  if (capacity < 0 || capacity > (int64_t)1 << 31) TCA_INVAL("capacity must be 0..2^31");
  tca_surrogate* s = new (std::nothrow) tca_surrogate;
  if (!s) {
    set_err("host allocation failed");
    return TCA_E_NOMEM;
  }
  s->Lc = Lc;
  s->dm = surrogate_dims(Lc, hidden);
  s->seed = seed;
  s->stream = (hipStream_t)hip_stream;
  s->capacity = capacity;
  const size_t np = s->dm.nparam;
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = s->W.alloc(np);
  if (e == hipSuccess) e = s->G.alloc(np);
  if (e == hipSuccess) e = s->m.alloc(np);
  if (e == hipSuccess) e = s->v.alloc(np);
  if (e == hipSuccess) e = s->W1b.alloc((size_t)hidden * s->dm.kpad);
  if (e == hipSuccess) e = s->W2b.alloc((size_t)hidden * hidden);
  if (e == hipSuccess && capacity > 0) e = s->X.alloc((size_t)capacity * s->dm.n_in);
  if (e == hipSuccess && capacity > 0) e = s->y.alloc((size_t)capacity);
  if (e == hipSuccess) e = sg_init_weights(s->W.p, s->dm, seed, s->stream);
  if (e == hipSuccess) e = sg_fill_f32(s->m.p, np, 0.0f, s->stream);
  if (e == hipSuccess) e = sg_fill_f32(s->v.p, np, 0.0f, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) {
    set_err("surrogate allocation failed: %s", hipGetErrorString(e));
    delete s;
    return e == hipErrorOutOfMemory ? TCA_E_NOMEM : TCA_E_DEVICE;
  }
  *out = s;
  return TCA_OK;
}

int tca_surrogate_destroy(tca_surrogate* s) {
  delete s;
  return TCA_OK;
}

int tca_surrogate_info(tca_surrogate* s, int64_t* nparams, int32_t* n_in, int64_t* rows) {
  g_err[0] = 0;
  if (!s) TCA_INVAL("NULL surrogate");
  if (nparams) *nparams = (int64_t)s->dm.nparam;
  if (n_in) *n_in = s->dm.n_in;
  if (rows) *rows = s->rows;
  return TCA_OK;
}

int tca_surrogate_save(tca_surrogate* s, float* params) {
  g_err[0] = 0;
  if (!s || !params) TCA_INVAL("NULL argument");
  TCA_CK(hipMemcpyAsync(params, s->W.p, sizeof(float) * s->dm.nparam, hipMemcpyDeviceToHost,
                        s->stream));
  TCA_CK(hipStreamSynchronize(s->stream));
  return TCA_OK;
}

int tca_surrogate_load(tca_surrogate* s, const float* params) {
  g_err[0] = 0;
  if (!s || !params) TCA_INVAL("NULL argument");
  for (size_t q = 0; q < s->dm.nparam; ++q)
    if (!isfinite(params[q])) TCA_INVAL("parameters must be finite");
  TCA_CK(hipMemcpyAsync(s->W.p, params, sizeof(float) * s->dm.nparam, hipMemcpyHostToDevice,
                        s->stream));
  TCA_CK(hipStreamSynchronize(s->stream));
  s->bf16_stale = true;
  return TCA_OK;
}

int tca_surrogate_collect(tca_surrogate* s, tca_ctx* c, const double* T, int32_t nsweeps,
                          tca_sweep_stats* st) {
  g_err[0] = 0;
  if (!s || !c) TCA_INVAL("NULL argument");
  const int rc = check_temps(T, nsweeps);
  if (rc != TCA_OK) return rc;
  if (c->p.n_classes != 0 || c->p.Lc != s->Lc)
    TCA_INVAL("collect needs a fixed cluster size equal to the surrogate's Lc");
  const int64_t need = (int64_t)nsweeps * c->N;
  if (need > s->capacity - s->rows) TCA_INVAL("dataset capacity exceeded");
  tca_surrogate* keep = c->sg;
  c->sg = nullptr;  // exact sweeps: the data must come from the plain chain
  const int r = run_sweeps(c, T, nsweeps, nullptr, st, s, s->rows);
  c->sg = keep;
  if (r == TCA_OK) s->rows += need;
  return r;
}

int tca_surrogate_get_rows(tca_surrogate* s, int64_t r0, int64_t rows, float* X, float* y) {
  g_err[0] = 0;
  if (!s || (rows > 0 && (!X || !y))) TCA_INVAL("NULL argument");
  if (r0 < 0 || rows < 0 || r0 + rows > s->rows) TCA_INVAL("rows outside the dataset");
  if (rows == 0) return TCA_OK;
  const int nin = s->dm.n_in;
  TCA_CK(hipMemcpyAsync(X, s->X.p + r0 * nin, sizeof(float) * rows * nin, hipMemcpyDeviceToHost,
                        s->stream));
  TCA_CK(hipMemcpyAsync(y, s->y.p + r0, sizeof(float) * rows, hipMemcpyDeviceToHost, s->stream));
  TCA_CK(hipStreamSynchronize(s->stream));
  return TCA_OK;
}

int tca_surrogate_add_rows(tca_surrogate* s, const float* X, const float* y, int64_t rows) {
  g_err[0] = 0;
  if (!s || (rows > 0 && (!X || !y))) TCA_INVAL("NULL argument");
  if (rows < 0 || rows > s->capacity - s->rows) TCA_INVAL("dataset capacity exceeded");
  if (rows == 0) return TCA_OK;
  const int nin = s->dm.n_in;
  TCA_CK(hipMemcpyAsync(s->X.p + s->rows * nin, X, sizeof(float) * rows * nin,
                        hipMemcpyHostToDevice, s->stream));
  TCA_CK(hipMemcpyAsync(s->y.p + s->rows, y, sizeof(float) * rows, hipMemcpyHostToDevice,
                        s->stream));
  TCA_CK(hipStreamSynchronize(s->stream));
  s->rows += rows;
  return TCA_OK;
}

int tca_surrogate_train(tca_surrogate* s, int32_t steps, int32_t batch, float lr, double holdout,
                        double* train_mse, double* rmse32, double* rmse16) {
  g_err[0] = 0;
  if (!s) TCA_INVAL("NULL surrogate");
  if (steps < 0 || batch < 1 || batch > (1 << 20)) TCA_INVAL("bad steps or batch");
  if (!(lr > 0.0f) || !isfinite(lr)) TCA_INVAL("lr must be finite and > 0");
  if (!(holdout >= 0.0 && holdout < 1.0)) TCA_INVAL("holdout must be in [0, 1)");
  const int64_t n_hold = (int64_t)floor(holdout * (double)s->rows);
  const int64_t n_train = s->rows - n_hold;
  if (steps > 0 && n_train < 1) TCA_INVAL("no training rows");
  // sized once for the minibatches and the held-out evaluation chunks
  if (ensure_train_bufs(s, batch > kEvalChunk ? batch : kEvalChunk) != hipSuccess) {
    set_err("training buffer allocation failed");
    return TCA_E_NOMEM;
  }
  if (steps > s->loss_cap) {
    TCA_CK(s->loss.alloc((size_t)steps));
    s->loss_cap = steps;
  }
  for (int k = 0; k < steps; ++k) {
    const SgTrainBufs b = train_bufs(s, s->loss.p + k);
    s->adam_t += 1;
    TCA_CK(sg_gather_batch(s->X.p, s->y.p, s->dm.n_in, 0, n_train, batch, s->seed,
                           (uint64_t)s->adam_t, b.Xb, b.yb, s->stream));
    TCA_CK(sg_forward_backward(s->W.p, s->dm, batch, b, s->G.p, s->stream));
    TCA_CK(sg_adam(s->W.p, s->G.p, s->m.p, s->v.p, s->dm.nparam, lr, s->adam_t, s->stream));
  }
  if (steps > 0) s->bf16_stale = true;
  if (train_mse) {
    *train_mse = 0.0;
    const int last = steps < 50 ? steps : 50;
    if (last > 0) {
      std::vector<double> h(last);
      TCA_CK(hipMemcpyAsync(h.data(), s->loss.p + (steps - last), sizeof(double) * last,
                            hipMemcpyDeviceToHost, s->stream));
      TCA_CK(hipStreamSynchronize(s->stream));
      for (double v : h) *train_mse += v / last;
    }
  }
  for (int q = 0; q < 2; ++q) {
    double* dst = q == 0 ? rmse32 : rmse16;
    if (!dst) continue;
    double sse = 0.0;
    const int r = holdout_sse(s, n_train, s->rows, q == 1, &sse);
    if (r != TCA_OK) return r;
    *dst = n_hold > 0 ? sqrt(sse / (double)n_hold) : 0.0;
  }
  TCA_CK(hipStreamSynchronize(s->stream));
  return TCA_OK;
}

int tca_surrogate_grad(tca_surrogate* s, const float* X, const float* y, int32_t rows,
                       float* grad, double* loss) {
  g_err[0] = 0;
  if (!s || !X || !y || !grad) TCA_INVAL("NULL argument");
  if (rows < 1 || rows > (1 << 20)) TCA_INVAL("rows must be 1..2^20");
  if (ensure_train_bufs(s, rows) != hipSuccess) {
    set_err("training buffer allocation failed");
    return TCA_E_NOMEM;
  }
  DevBuf<double> dl;
  TCA_CK(dl.alloc(1));
  const SgTrainBufs b = train_bufs(s, dl.p);
  TCA_CK(hipMemcpyAsync(b.Xb, X, sizeof(float) * rows * s->dm.n_in, hipMemcpyHostToDevice,
                        s->stream));
  TCA_CK(hipMemcpyAsync(b.yb, y, sizeof(float) * rows, hipMemcpyHostToDevice, s->stream));
  TCA_CK(sg_forward_backward(s->W.p, s->dm, rows, b, s->G.p, s->stream));
  TCA_CK(hipMemcpyAsync(grad, s->G.p, sizeof(float) * s->dm.nparam, hipMemcpyDeviceToHost,
                        s->stream));
  double l = 0.0;
  TCA_CK(hipMemcpyAsync(&l, dl.p, sizeof(double), hipMemcpyDeviceToHost, s->stream));
  TCA_CK(hipStreamSynchronize(s->stream));
  if (loss) *loss = l;
  return TCA_OK;
}

int tca_surrogate_adam_step(tca_surrogate* s, const float* grad, float lr) {
  g_err[0] = 0;
  if (!s || !grad) TCA_INVAL("NULL argument");
  if (!(lr > 0.0f) || !isfinite(lr)) TCA_INVAL("lr must be finite and > 0");
  TCA_CK(hipMemcpyAsync(s->G.p, grad, sizeof(float) * s->dm.nparam, hipMemcpyHostToDevice,
                        s->stream));
  s->adam_t += 1;
  TCA_CK(sg_adam(s->W.p, s->G.p, s->m.p, s->v.p, s->dm.nparam, lr, s->adam_t, s->stream));
  TCA_CK(hipStreamSynchronize(s->stream));
  s->bf16_stale = true;
  return TCA_OK;
}

int tca_surrogate_eval(tca_surrogate* s, const float* X, int32_t rows, int32_t bf16, float* out) {
  g_err[0] = 0;
  if (!s || !X || !out) TCA_INVAL("NULL argument");
  if (rows < 0 || rows > (1 << 24)) TCA_INVAL("rows must be 0..2^24");
  if (bf16 != 0 && bf16 != 1) TCA_INVAL("bf16 must be 0 or 1");
  if (rows == 0) return TCA_OK;
  const int nin = s->dm.n_in, H = s->dm.hidden;
  DevBuf<float> dX, dout;
  TCA_CK(dX.alloc((size_t)rows * nin));
  TCA_CK(dout.alloc((size_t)rows));
  TCA_CK(hipMemcpyAsync(dX.p, X, sizeof(float) * rows * nin, hipMemcpyHostToDevice, s->stream));
  if (bf16) {
    DevBuf<uint16_t> Fb, H1, H2;
    TCA_CK(Fb.alloc((size_t)rows * s->dm.kpad));
    TCA_CK(H1.alloc((size_t)rows * H));
    TCA_CK(H2.alloc((size_t)rows * H));
    if (s->bf16_stale) {
      TCA_CK(sg_to_bf16(s->W.p, s->dm, s->W1b.p, s->W2b.p, s->stream));
      s->bf16_stale = false;
    }
    TCA_CK(sg_f32_to_bf16_rows(dX.p, rows, nin, s->dm.kpad, Fb.p, s->stream));
    TCA_CK(sg_infer_bf16(Fb.p, rows, s->W.p, s->W1b.p, s->W2b.p, s->dm, SgInferBufs{H1.p, H2.p},
                         dout.p, s->stream));
    TCA_CK(hipMemcpyAsync(out, dout.p, sizeof(float) * rows, hipMemcpyDeviceToHost, s->stream));
    TCA_CK(hipStreamSynchronize(s->stream));
  } else {
    DevBuf<float> z1, h1, z2, h2;
    TCA_CK(z1.alloc((size_t)rows * H));
    TCA_CK(h1.alloc((size_t)rows * H));
    TCA_CK(z2.alloc((size_t)rows * H));
    TCA_CK(h2.alloc((size_t)rows * H));
    SgTrainBufs b{dX.p, nullptr, z1.p, h1.p, z2.p, h2.p, dout.p,
                  nullptr, nullptr, nullptr, nullptr, nullptr};
    TCA_CK(sg_forward(s->W.p, s->dm, rows, b, s->stream));
    TCA_CK(hipMemcpyAsync(out, dout.p, sizeof(float) * rows, hipMemcpyDeviceToHost, s->stream));
    TCA_CK(hipStreamSynchronize(s->stream));
  }
  return TCA_OK;
}

int tca_attach_surrogate(tca_ctx* c, tca_surrogate* s) {
  g_err[0] = 0;
  if (!c) TCA_INVAL("NULL context");
  if (!s) {
    c->sg = nullptr;
    return TCA_OK;
  }
  if (c->p.n_classes != 0) {
    set_err("delayed acceptance needs a fixed cluster size");
    return TCA_E_UNSUPPORTED;
  }
  if (c->p.Lc != s->Lc) TCA_INVAL("surrogate and context cluster sizes differ");
  const int hh = c->h * c->h;
  if (c->da.rows != 2 * hh) {
    DaBufs& d = c->da;
    TCA_CK(d.Fin.alloc((size_t)2 * hh * s->dm.kpad));
    TCA_CK(d.dS.alloc((size_t)2 * hh));
    TCA_CK(d.pass.alloc((size_t)hh));
    TCA_CK(d.count.alloc(1));
    TCA_CK(d.list.alloc((size_t)hh));
    d.rows = 2 * hh;
  }
  // hidden activations follow the surrogate's width
  TCA_CK(c->da.H1.alloc((size_t)2 * hh * s->dm.hidden));
  TCA_CK(c->da.H2.alloc((size_t)2 * hh * s->dm.hidden));
  c->sg = s;
  return TCA_OK;
}

}  // extern "C"
